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
// block scan for every byte's output position; then each thread builds 16
// bytes of the destination from those positions and stores them at once.
// Large jobs size every tile first, scan the tile totals and then emit at
// known offsets, so that no workgroup waits for another.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <stddef.h>
#include <tuple>
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

constexpr int kCL = 256;              // lines per tile at most (one per thread)
// LDS bytes of a batch's raw lines (reused as output stage) and, as many, of
// their pre-processed form: the default variant runs 3 workgroups per CU, the
// large one (long lines) 2.
constexpr int kCapSmall = 14336;
// binned short bins: a tile of 256 bulk lines (13.2 KB on average) fits one batch,
// and with the default dictionary three workgroups (ABS array included) fit a CU
constexpr int kCapGather = 15360;
constexpr int kCapLarge = 26624;
// Global-memory layout (long-line bins): the line buffers of a workgroup live in
// its own region of the workspace, so LDS holds only the automaton and the
// per-line arrays and a tile of 256 long lines keeps every lane busy.
constexpr int kCapGlobal = 262144;
constexpr size_t kGlStride = 2 * (size_t)kCapGlobal + kCapGlobal / 8 + 256;  // RAW, PRE, ESC bits, margins
// Global-memory layout: the ring pass's LDS tables, per lane: a byte per label
// value (its open ring's slot + 1) and kOpenSlots u16 slots of open rings.  They
// share LDS with the dictionary image, which is staged again before the parse.
constexpr int kLabels = 100;
constexpr int kOpenSlots = 32;
constexpr uint32_t kRingRegion = (uint32_t)(kLabels + 2 * kOpenSlots) * 256u;
constexpr int kSlots = 8;             // fast ring table (registers): up to 8 open rings, found by label
constexpr int kSlotsFirst = 4;        // the smaller table tried first
constexpr int kGenLane = 400;         // per-lane ring tables in global memory (any line):
                                      // 100 open positions u16 + 100 last-close u16
static_assert(kCapGather >= 3 * (int)ZS_MAX_LINE, "a pre-processed line must fit");
static_assert(kCapGather >= (int)ZS_MAX_LINE + 1 + 16, "a raw line must fit");
constexpr uint64_t kAbsBad = 1ull << 63;  // ABS flag (binned mode): the line's framing is bad

// What a compression launch writes: compressed lines, or only the lines with
// their rings relabelled - by the pre-processing rule (Sec. IV-A) or by the
// post-processing rule (zs_postprocess).
constexpr int kModeCompress = 0, kModePre = 1, kModePost = 2;
constexpr uint8_t kSkip = 0x7F;    // marker: byte dropped by pre-processing
constexpr uint8_t kIdMark = 0x80;  // marker: ring-label with ID (low 7 bits)
constexpr uint32_t kBadLine = 0x8000u;  // LENS flag: the line is bad (empty output)

struct CompressLds {
    uint32_t tab_bytes;  // dictionary part staged
    uint32_t raw, pre, esc, off, cost, eoff, lens, perm, misc, sink, ident, ring, eri, abs;
    uint32_t total;         // plain mode
    uint32_t total_gather;  // binned mode (ABS at the end)
};

__host__ __device__ inline CompressLds compress_lds(uint32_t tab_bytes, uint32_t cap, bool gl = false) {
    CompressLds L;
    L.tab_bytes = align16(tab_bytes);
    // gl: the dictionary's region also holds the ring tables, then the expansion
    // rings; the emission rings follow the dictionary
    L.ring = 0;
    L.eri = L.tab_bytes;
    const uint32_t gl_region = L.tab_bytes + kCL * 32 > kRingRegion ? L.tab_bytes + kCL * 32 : kRingRegion;
    uint32_t o = gl ? gl_region : L.tab_bytes;
    const uint32_t lds_cap = gl ? 0u : cap;  // gl: RAW, PRE and ESC are in global memory
    L.raw = o;  o += lds_cap;
    L.pre = o;  o += lds_cap;
    L.esc = o;  o += lds_cap / 8;
    L.off = o;  o += align16((kCL + 1) * 8);
    L.cost = o; o += kCL * 4;
    L.eoff = o; o += kCL * 4;
    L.lens = o; o += kCL * 2;
    L.perm = o; o += kCL * 2;
    L.misc = o; o += 256;
    L.sink = o; o += kCL;  // one byte per lane: stores of parse steps past the line's start
    L.ident = o; o += 256; // ident[b] = b: an escaped byte is looked up like a code
    L.total = align16(o);
    L.abs = L.total;  // only binned launches allocate it
    L.total_gather = L.abs + align16(kCL * 8);
    return L;
}

// Tile geometry of the length bins (binned mode), written on the device.
// Bins are numbered in the order they are processed: longest lines first.
constexpr int kMaxBins = 8;
struct BinPlan {
    uint32_t nbins;
    uint32_t upper[kMaxBins];          // bin b holds lines of raw length < upper[b] (and >= upper[b + 1])
    uint32_t lpt[kMaxBins];            // lines per tile of bin b
    uint32_t count[kMaxBins];          // lines in bin b
    uint64_t start[kMaxBins];          // first position of bin b in the id order
    uint32_t first_tile[kMaxBins + 1]; // global index of bin b's first tile; [nbins] = all tiles
    uint32_t ticket[kMaxBins];         // per-launch tile counters
};

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
    uint8_t* slots;         // CAP bytes per workgroup: a finished tile waiting for its offset
    // binned mode (null ids: plain mode, tile t = lines [256 t, 256 t + 256))
    const uint32_t* ids;    // line ids in bin order
    const struct BinPlan* plan;
    uint32_t bin_lo, bin_hi;  // the bins this launch takes
    uint32_t* ticket;       // this launch's tile counter
    uint8_t* glines;        // global-memory layout: kGlStride bytes per workgroup
};

__device__ inline bool is_digit(uint32_t c) { return c - '0' < 10u; }

// Per-lane state of the line a lane holds inside a batch.
struct LineState {
    uint32_t j;     // line index inside the batch (lanes are assigned by length rank)
    uint32_t R;     // raw offset in RAW
    uint32_t len;   // raw length (newline excluded)
    uint32_t m;     // pre-processed length (0 for a bad line)
    uint32_t P;     // offset in PRE
    bool in;        // this lane holds a line of the batch
    bool bad;       // framing or byte error: the output line is empty
    bool simple;    // batch-wide: no line changed length, tokens live in RAW, stage is PRE
    bool esc;       // batch-wide: some byte was escaped (the ESC bits are needed)
};

__device__ inline void restore_line(uint8_t* raw, uint32_t R, const uint8_t* src, uint32_t len) {
    for (uint32_t i = 0; i < len; i++) raw[R + i] = src[i];
}

// Ring IDs of one line with tables in global memory (any number of rings and
// IDs): the rule of Sec. IV-A written as "latest close per ID": a closing ring
// takes the smallest ID whose latest closing label precedes its opening label.
// post: the post-processing rule instead - an opening ring takes the smallest
// label >= 1 not held by an open ring (last[v] then holds the label of the
// open ring of value v).  Markers are written over the raw line.  Returns
// false if the line is malformed or needs an ID of 100 or more (the raw bytes
// are then partly overwritten and must be restored).
template <bool post>
__device__ inline bool ring_general(uint8_t* raw, uint32_t R, uint32_t len, uint16_t* open, uint16_t* last,
                                    int* delta) {
    for (int k = 0; k < 100; k++) { open[k] = 0; last[k] = 0; }
    uint64_t held0 = 1, held1 = 0;  // post: labels held by open rings (label 0 is never used)
    int dl = 0, opens = 0;
    uint32_t inbr = 0;
    for (uint32_t i = 0; i < len; i++) {
        const uint32_t c = raw[R + i];
        if (c == '[') { inbr = 1; continue; }
        if (c == ']') { inbr = 0; continue; }
        if (inbr) continue;
        uint32_t v, tl;
        if (is_digit(c)) { v = c - '0'; tl = 1; }
        else if (c == '%') { v = (raw[R + i + 1] - '0') * 10u + (raw[R + i + 2] - '0'); tl = 3; }
        else continue;
        const uint32_t e = open[v];
        if (e == 0) {
            open[v] = (uint16_t)(i + 1);
            opens++;
            if constexpr (post) {
                uint32_t l = 1;
                while (l < 100 && ((l < 64 ? held0 >> l : held1 >> (l - 64)) & 1u)) l++;
                if (l >= 100) return false;
                if (l < 64) held0 |= 1ull << l;
                else held1 |= 1ull << (l - 64);
                last[v] = (uint16_t)l;
            }
        } else {
            const uint32_t o = e - 1;
            open[v] = 0;
            opens--;
            uint32_t id = 0;
            if constexpr (post) {
                id = last[v];
                if (id < 64) held0 &= ~(1ull << id);
                else held1 &= ~(1ull << (id - 64));
            } else {
                while (id < 100 && (uint32_t)last[id] > o + 1) id++;
                if (id >= 100) return false;
                last[id] = (uint16_t)(i + 1);
            }
            const uint32_t to = (raw[R + o] == '%') ? 3u : 1u;
            raw[R + o] = (uint8_t)(kIdMark | id);
            if (to == 3) raw[R + o + 1] = raw[R + o + 2] = kSkip;
            raw[R + i] = (uint8_t)(kIdMark | id);
            if (tl == 3) raw[R + i + 1] = raw[R + i + 2] = kSkip;
            const int nlen = id < 10 ? 1 : 3;
            dl += (nlen - (int)to) + (nlen - (int)tl);
        }
        i += tl - 1;
    }
    *delta = dl;
    return opens == 0;
}

template <int LK, int CAP, int MODE, bool GL = false>
struct Compressor {
    static constexpr int kRawCap = CAP, kPreCap = CAP, kSlotBytes = CAP;
    const CompressArgs A;
    uint8_t* smem;
    CompressLds L;
    uint8_t* g_raw = nullptr;  // GL: this workgroup's line buffers in global memory
    uint8_t* g_pre = nullptr;
    uint32_t* g_esc = nullptr;
    const TableHeader* H;
    const uint8_t* LENT;  // expansion lengths
    const uint8_t* COL;
    const uint16_t* TRANS;
    const uint8_t* OUTK;  // signed bytes, LK per state
    uint32_t off_code1, off_code;
    uint32_t C;  // automaton columns

    __device__ Compressor(const CompressArgs& a, uint8_t* s) : A(a), smem(s) {
        L = compress_lds(a.tab_bytes, CAP, GL);
        if constexpr (GL) {
            uint8_t* b = a.glines + (uint64_t)blockIdx.x * kGlStride + 128;
            g_raw = b;
            g_pre = b + CAP;
            g_esc = (uint32_t*)(b + 2 * (size_t)CAP);
        }
        H = (const TableHeader*)smem;
        if constexpr (MODE == kModeCompress) {
            LENT = smem + H->off_len;
            COL = smem + H->off_col;
            TRANS = (const uint16_t*)(smem + H->off_trans);
            OUTK = smem + H->off_outk;
            off_code1 = H->off_code1;
            off_code = H->off_code;
            C = H->ncols;
        } else {  // pre-processing only: no dictionary staged, none read
            LENT = COL = nullptr;
            TRANS = nullptr;
            OUTK = nullptr;
            off_code1 = off_code = C = 0;
        }
    }

    __device__ __forceinline__ uint64_t* OFF() { return (uint64_t*)(smem + L.off); }
    __device__ __forceinline__ uint64_t* ABS() { return (uint64_t*)(smem + L.abs); }
    __device__ __forceinline__ uint32_t* COST() { return (uint32_t*)(smem + L.cost); }
    __device__ __forceinline__ uint32_t* EOFF() { return (uint32_t*)(smem + L.eoff); }
    __device__ __forceinline__ uint16_t* LENS() { return (uint16_t*)(smem + L.lens); }
    __device__ __forceinline__ uint16_t* PERM() { return (uint16_t*)(smem + L.perm); }
    __device__ __forceinline__ uint32_t* MISC() { return (uint32_t*)(smem + L.misc); }
    __device__ __forceinline__ uint8_t* RAW() {
        if constexpr (GL) return g_raw;
        else return smem + L.raw;
    }
    __device__ __forceinline__ uint8_t* PRE() {
        if constexpr (GL) return g_pre;
        else return smem + L.pre;
    }
    __device__ __forceinline__ uint32_t* ESC() {
        if constexpr (GL) return g_esc;
        else return (uint32_t*)(smem + L.esc);
    }
    // Workgroup barrier.  GL: a barrier does not wait for a wave's global stores,
    // and the line buffers are written by one wave and read by another, so
    // every wave first waits for its own memory operations to complete.
    __device__ __forceinline__ void bar() {
        if constexpr (GL) __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    __device__ __forceinline__ bool bar_or(bool v) {
        if constexpr (GL) __builtin_amdgcn_s_waitcnt(0);
        return __syncthreads_or(v) != 0;
    }
    __device__ __forceinline__ bool bar_and(bool v) {
        if constexpr (GL) __builtin_amdgcn_s_waitcnt(0);
        return __syncthreads_and(v) != 0;
    }

    // Index of line j of the tile in the input (binned mode: from the id list).
    __device__ __forceinline__ uint64_t line_id(uint64_t k0, uint32_t j) { return A.ids ? A.ids[k0 + j] : k0 + j; }
    // Input bytes of line j of the tile.
    __device__ __forceinline__ const uint8_t* line_src(uint32_t j) {
        return A.in + (A.ids ? (ABS()[j] & ~kAbsBad) : OFF()[j]);
    }

    // Framing of line j of the tile (OFF staged).  0 = ok, else error kind.
    __device__ __forceinline__ uint32_t frame_error(uint64_t k0, uint32_t j) {
        if (A.ids) return (ABS()[j] & kAbsBad) ? kErrInval : 0u;
        const uint64_t a = OFF()[j], b = OFF()[j + 1];
        if (b <= a || b > A.in_bytes + 1) return kErrInval;
        if (b - a - 1 > ZS_MAX_LINE) return kErrInval;
        if (b == A.in_bytes + 1 && k0 + j + 1 != A.n) return kErrInval;
        return 0;
    }

    // Forward scan of one raw line, four bytes at a time with byte-parallel
    // masks (one flag bit per byte, at bit 7 of each byte): bad bytes, bracket
    // depth, ring labels - a digit outside brackets, or '%' outside brackets
    // followed by two digits (Sec. II).  Labels go to `list`: u16 entries hold
    // the position in the line << 4 and the digit, or 15 for a '%' label; u32
    // entries (global-memory layout: list 16-byte aligned, stored four entries
    // at a time) the position << 8, 0x80 for a '%' label and the label value.
    __device__ static inline uint32_t eq_bytes(uint32_t w, uint32_t pat) {
        const uint32_t x = w ^ pat;
        return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
    }
    template <typename E>
    __device__ __forceinline__ void scan_labels(const uint8_t* raw, uint32_t R, uint32_t len, E* list, uint32_t cap,
                                uint32_t* nlab_out, bool* corrupt_out, bool* malformed_out, bool* over_out,
                                bool* has_pct) {
        uint32_t inbr = 0;      // bracket state before the current word (0 or 0x80808080-style all-ones flag)
        uint32_t carry = 0;     // bytes of this word consumed by a '%' of the previous word (flag bits)
        uint32_t nlab = 0;
        uint32_t bad = 0, mal = 0, pct_any = 0;
        bool over = false;
        const uint32_t end = R + len;
        // u32 entries: queued in LDS (16 per lane, dword-interleaved, in the ring
        // tables' slot area: the caller's barrier ends every scan before any ring pass)
        uint32_t* eq = (uint32_t*)(smem + L.ring + kLabels * kWG) + threadIdx.x;
        // one word: w its position (w < end), next the word after it
        auto step = [&](uint32_t w, uint32_t word, uint32_t next) __attribute__((always_inline)) {
            // flag bits of the bytes of this word that belong to the line
            // (clamps in signed arithmetic: see the note at the decoder's valid mask)
            const uint32_t lo = (uint32_t)min(max((int32_t)R - (int32_t)w, 0), 4), hi = min(end - w, 4u);
            const uint32_t inl = lo >= 4 ? 0u : (0x80808080u << (8 * lo)) & (0x80808080u >> (8 * (4 - hi)));
            const uint32_t nhi = (uint32_t)min(max((int32_t)end - (int32_t)w - 4, 0), 4);
            const uint32_t inl_n = nhi ? (0x80808080u >> (8 * (4 - nhi))) : 0u;
            // byte classes (valid only for bytes < 0x80; other bytes are corrupt anyway)
            const uint32_t ge30 = ((word & 0x7F7F7F7Fu) + 0x50505050u) & 0x80808080u;
            const uint32_t ge3a = ((word & 0x7F7F7F7Fu) + 0x46464646u) & 0x80808080u;
            const uint32_t dig = ge30 & ~ge3a & ~word & inl;
            const uint32_t ge20 = ((word & 0x7F7F7F7Fu) + 0x60606060u) & 0x80808080u;
            bad |= ((word & 0x80808080u) | (~ge20 & 0x80808080u) | eq_bytes(word, 0x7F7F7F7Fu)) & inl;
            const uint32_t op = eq_bytes(word, 0x5B5B5B5Bu) & inl;   // '['
            const uint32_t cl = eq_bytes(word, 0x5D5D5D5Du) & inl;   // ']'
            const uint32_t pc = eq_bytes(word, 0x25252525u) & inl;   // '%'
            const uint32_t ge30n = ((next & 0x7F7F7F7Fu) + 0x50505050u) & 0x80808080u;
            const uint32_t ge3an = ((next & 0x7F7F7F7Fu) + 0x46464646u) & 0x80808080u;
            const uint32_t dign = ge30n & ~ge3an & ~next & inl_n;
            // bracket state before each byte: prefix parity of the bracket bytes
            const uint32_t br = op | cl;
            uint32_t px = br ^ (br << 8);
            px ^= px << 16;                      // inclusive prefix xor
            const uint32_t inside = (px ^ br) ^ inbr;   // before each byte
            mal |= (op & inside) | (cl & ~inside & 0x80808080u);
            inbr = (px & 0x80000000u) ? (inbr ^ 0x80808080u) : inbr;
            // '%' outside brackets must be followed by two digits, which it consumes
            const uint32_t pco = pc & ~inside;
            const uint64_t d64 = (uint64_t)dig | ((uint64_t)dign << 32);
            const uint64_t need = ((uint64_t)pco << 8) | ((uint64_t)pco << 16);
            mal |= (uint32_t)((need & ~d64) != 0);
            const uint32_t consumed = (uint32_t)need | carry;
            carry = (uint32_t)(need >> 32);
            pct_any |= pco;
            const uint32_t lab = ((dig & ~inside & ~consumed) | pco) & 0x80808080u;
            const uint32_t n0 = nlab;
            if (lab) {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    if (lab & (0x80u << (8 * k))) {
                        const uint32_t cb = (word >> (8 * k)) & 0xFFu;
                        uint32_t ent;
                        if constexpr (sizeof(E) == 2) {
                            ent = ((w + k - R) << 4) | ((cb == '%') ? 15u : cb - '0');
                        } else {
                            // a '%' label's two digits are in this word or the next
                            const uint64_t wn = (uint64_t)word | ((uint64_t)next << 32);
                            const uint32_t d1 = (uint32_t)(wn >> (8 * (k + 1))) & 0xFFu;
                            const uint32_t d2 = (uint32_t)(wn >> (8 * (k + 2))) & 0xFFu;
                            ent = ((w + k - R) << 8) |
                                  ((cb == '%') ? (0x80u | (((d1 - '0') * 10u + (d2 - '0')) & 0x7Fu)) : cb - '0');
                        }
                        if constexpr (sizeof(E) == 2) {
                            if (nlab < cap) list[nlab] = (E)ent;
                            else over = true;
                        } else {
                            eq[(nlab & 15u) * kWG] = ent;
                        }
                        nlab++;
                    }
                }
            }
            if constexpr (sizeof(E) == 4) {
                // a word completes at most one group
                const uint32_t g = n0 >> 2;
                if ((nlab >> 2) != g && 4 * g + 4 <= cap) {
                    const uint32_t* e4 = eq + ((4 * g) & 15u) * kWG;
                    *(uint4*)(list + 4 * g) = make_uint4(e4[0], e4[kWG], e4[2 * kWG], e4[3 * kWG]);
                }
            }
        };
        if constexpr (sizeof(E) == 4) {
            // global-memory layout: 16-byte loads, one chunk in flight ahead
            const uint32_t c0 = R & ~15u;
            uint4 cu = *(const uint4*)(raw + c0);
            uint4 nx = *(const uint4*)(raw + c0 + 16);
            for (uint32_t c = c0; c < end; c += 16) {
                const uint4 n2 = *(const uint4*)(raw + c + 32);  // at most 47 bytes past the line: in the buffer
                step(c, cu.x, cu.y);
                if (c + 4 < end) step(c + 4, cu.y, cu.z);
                if (c + 8 < end) step(c + 8, cu.z, cu.w);
                if (c + 12 < end) step(c + 12, cu.w, nx.x);
                cu = nx;
                nx = n2;
            }
            const uint32_t g = nlab >> 2;
            if ((nlab & 3u) && 4 * g + 4 <= cap) {  // the last, partial group
                const uint32_t* e4 = eq + ((4 * g) & 15u) * kWG;
                *(uint4*)(list + 4 * g) = make_uint4(e4[0], e4[kWG], e4[2 * kWG], e4[3 * kWG]);
            }
            over = nlab > cap;
        } else {
            const uint32_t w0 = R & ~3u;
            // two words in flight ahead of the one being classified
            uint32_t word = *(const uint32_t*)(raw + w0);
            uint32_t next = *(const uint32_t*)(raw + w0 + 4);
            for (uint32_t w = w0; w < end; w += 4) {
                const uint32_t next2 = *(const uint32_t*)(raw + w + 8);
                step(w, word, next);
                word = next;
                next = next2;
            }
        }
        *nlab_out = nlab;
        *corrupt_out = bad != 0;
        *malformed_out = (mal != 0) | (inbr != 0);
        *over_out = over;
        *has_pct = pct_any != 0;
    }

    // Ring IDs from the label list with a register table of NS open rings
    // (found by label value, free slots reused) and, per open ring, the bit set
    // of the IDs of the rings that closed inside it; a closing ring takes the
    // smallest ID not in its set (Sec. IV-A).  post: the post-processing rule
    // instead - an opening ring takes the smallest label >= 1 not held by an
    // open ring, kept in the ring's word of the set table.  Markers are written
    // over the raw line.  Sets *overflow when more than NS rings are open at
    // once or an ID reaches 32; returns false when rings stay open.
    template <int NS, bool post>
    __device__ __forceinline__ bool ring_fast(uint8_t* raw, uint32_t R, const uint16_t* list, uint32_t nlab, uint32_t maxlab,
                              int* delta, bool* overflow, bool* marked) {
        // slot word of an open ring: (position + 1) << 8 | ('%' label) << 7 | label
        bool mk_any = false;
        uint32_t os[NS], mk[NS];
#pragma unroll
        for (int k = 0; k < NS; k++) { os[k] = 0; mk[k] = 0; }
        uint32_t held = 1u;  // post: labels held by open rings (label 0 is never used)
        int dl = 0, opens = 0;
        bool ovf = false;
        uint32_t nxt = list[0];
        for (uint32_t q = 0; q < maxlab; q++) {
            const uint32_t ent = nxt;
            nxt = list[q + 1];  // next entry ahead of time (past the end: unused bytes of PRE)
            if (q < nlab && !ovf) {
                const uint32_t p = ent >> 4;
                uint32_t v, tl;
                if ((ent & 15u) == 15u) {
                    v = (raw[R + p + 1] - '0') * 10u + (raw[R + p + 2] - '0');
                    tl = 3;
                } else {
                    v = ent & 15u;
                    tl = 1;
                }
                // the open ring of label v, else the first free slot
                uint32_t slot = NS, freeslot = NS;
#pragma unroll
                for (int k = NS - 1; k >= 0; k--) {
                    slot = (os[k] != 0 && (os[k] & 0x7Fu) == v) ? (uint32_t)k : slot;
                    freeslot = (os[k] == 0) ? (uint32_t)k : freeslot;
                }
                uint32_t e = 0, m = 0;
                if (slot == NS) {
                    slot = freeslot;
                } else {
#pragma unroll
                    for (int k = 0; k < NS; k++) {
                        e = (slot == (uint32_t)k) ? os[k] : e;
                        m = (slot == (uint32_t)k) ? mk[k] : m;
                    }
                }
                if (slot == NS) {
                    ovf = true;  // more than NS rings open
                } else if (e == 0) {
                    // post: the opening takes the smallest free label (at most NS are held)
                    const uint32_t nl = post ? (uint32_t)__builtin_ctz(~held) : 0u;
                    held |= post ? (1u << nl) : 0u;
#pragma unroll
                    for (int k = 0; k < NS; k++) {
                        os[k] = (slot == (uint32_t)k) ? (((p + 1) << 8) | (tl == 3 ? 0x80u : 0u) | v) : os[k];
                        mk[k] = (slot == (uint32_t)k) ? nl : mk[k];
                    }
                    opens++;
                } else if ((e & 0x7Fu) == v) {
                    const uint32_t o = (e >> 8) - 1;
                    const uint32_t id = post ? m : (uint32_t)__builtin_ctz(~m);
                    if (!post && m == 0xFFFFFFFFu) {
                        ovf = true;
                    } else {
                        const uint32_t bit = 1u << id;
                        held &= post ? ~bit : ~0u;
#pragma unroll
                        for (int k = 0; k < NS; k++) {
                            os[k] = (slot == (uint32_t)k) ? 0u : os[k];
                            mk[k] |= post ? 0u : bit;
                        }
                        opens--;
                        const uint32_t to = (e & 0x80u) ? 3u : 1u;
                        const int nlen = id < 10 ? 1 : 3;
                        // a one-byte label that stays one byte takes its new digit in place;
                        // anything else is marked for the expansion pass
                        const uint8_t nb = (nlen == 1) ? (uint8_t)('0' + id) : (uint8_t)(kIdMark | id);
                        raw[R + o] = (to == 1) ? nb : (uint8_t)(kIdMark | id);
                        if (to == 3) raw[R + o + 1] = raw[R + o + 2] = kSkip;
                        raw[R + p] = (tl == 1) ? nb : (uint8_t)(kIdMark | id);
                        if (tl == 3) raw[R + p + 1] = raw[R + p + 2] = kSkip;
                        mk_any |= (nlen != 1) | (to != 1) | (tl != 1);
                        dl += (nlen - (int)to) + (nlen - (int)tl);
                    }
                }
            }
        }
        *delta = dl;
        *overflow = ovf;
        *marked = mk_any;
        return opens == 0;
    }

    // Ring IDs of the global-memory layout (long lines, many rings open at once):
    // the rule of Sec. IV-A as "latest close per ID", like ring_general, from
    // the u32 label list (16-byte aligned, read four entries at a time).  In LDS,
    // per lane: the label byte of value v holds its open ring's slot + 1 (0 when
    // closed; cleared by the caller), a slot the opening position + 1 and 0x8000
    // for a '%' label; in registers the free slots and the latest closing
    // position of IDs 0..31.  A closing writes one byte at each of the two
    // labels: the new digit when a one-byte label stays one byte, else a marker
    // 0x80 | id with 0x40 set when the label was a '%' label (the expansion then
    // drops its two digits).  Sets *overflow when more than kOpenSlots rings are
    // open or an ID reaches 32 (the caller restores the line and takes
    // ring_general); returns false when rings stay open.
    __device__ __forceinline__ bool ring_table(uint8_t* raw, uint32_t R, const uint32_t* list, uint32_t nlab,
                                               uint32_t maxlab, int* delta, bool* overflow, bool* marked) {
        uint8_t* tab = smem + L.ring + threadIdx.x;                                      // label v at tab[v * kWG]
        uint16_t* slots = (uint16_t*)(smem + L.ring + kLabels * kWG) + threadIdx.x;  // slot k at slots[k * kWG]
        uint32_t used = 0;  // open slots
        uint32_t lct[32];   // closing position + 1 of the latest ring that took ID k; 0: none
#pragma unroll
        for (int k = 0; k < 32; k++) lct[k] = 0;
        bool mk_any = false, ovf = false;
        int dl = 0, opens = 0;
        auto label = [&](uint32_t ent, uint32_t q) __attribute__((always_inline)) {
            if (q >= nlab || ovf) return;
            const uint32_t v = min(ent & 0x7Fu, (uint32_t)kLabels - 1);
            const uint32_t p = (ent >> 8) & 0xFFFu;
            const uint32_t tl = (ent & 0x80u) ? 3u : 1u;
            const uint32_t t = tab[v * kWG];
            if (t == 0) {
                if (used == 0xFFFFFFFFu) {
                    ovf = true;
                    return;
                }
                const uint32_t k = (uint32_t)__builtin_ctz(~used);
                used |= 1u << k;
                slots[k * kWG] = (uint16_t)((p + 1) | (tl == 3 ? 0x8000u : 0u));
                tab[v * kWG] = (uint8_t)(k + 1);
                opens++;
                return;
            }
            if (t > (uint32_t)kOpenSlots || !((used >> (t - 1)) & 1u)) {  // not a ring of this pass
                ovf = true;
                return;
            }
            const uint32_t cur = slots[(t - 1) * kWG];
            const uint32_t o = (cur & 0x7FFFu) - 1;
            // IDs taken by a ring that closed after this one opened
            uint32_t M = 0;
#pragma unroll
            for (int k = 31; k >= 0; k--) M = (M << 1) | (lct[k] > o + 1 ? 1u : 0u);
            if (M == 0xFFFFFFFFu) {
                ovf = true;
                return;
            }
            const uint32_t id = (uint32_t)__builtin_ctz(~M);
#pragma unroll
            for (int k = 0; k < 32; k++) lct[k] = ((uint32_t)k == id) ? p + 1 : lct[k];
            used &= ~(1u << (t - 1));
            tab[v * kWG] = 0;
            opens--;
            const uint32_t to = (cur & 0x8000u) ? 3u : 1u;
            const int nlen = id < 10 ? 1 : 3;
            raw[R + o] = (to == 1 && nlen == 1) ? (uint8_t)('0' + id) : (uint8_t)(kIdMark | (to == 3 ? 0x40u : 0u) | id);
            raw[R + p] = (tl == 1 && nlen == 1) ? (uint8_t)('0' + id) : (uint8_t)(kIdMark | (tl == 3 ? 0x40u : 0u) | id);
            mk_any |= (nlen != 1) | (to != 1) | (tl != 1);
            dl += (nlen - (int)to) + (nlen - (int)tl);
        };
        // two groups of four entries in flight; a group is reloaded right after its use
        const uint4* l4 = (const uint4*)list;  // entries past the end: unused bytes of PRE, never processed
        uint4 ga = l4[0], gb = l4[1];
        for (uint32_t q0 = 0; q0 < maxlab; q0 += 8) {
            label(ga.x, q0);
            label(ga.y, q0 + 1);
            label(ga.z, q0 + 2);
            label(ga.w, q0 + 3);
            ga = l4[(q0 >> 2) + 2];
            if (q0 + 4 >= maxlab) break;
            label(gb.x, q0 + 4);
            label(gb.y, q0 + 5);
            label(gb.z, q0 + 6);
            label(gb.w, q0 + 7);
            gb = l4[(q0 >> 2) + 3];
        }
        *delta = dl;
        *overflow = ovf;
        *marked = mk_any;
        return opens == 0;
    }

    struct ParseState {
        uint32_t V[LK];  // (cost + 1) << 5 of the next LK positions, in rotating slots
        uint32_t s;      // automaton state after the current byte
        uint32_t c;      // current byte
        uint32_t cn, coln;  // the byte before it and its column
    };

    // Steps K.. of one unrolled group: at step K the cost of position i+L sits in
    // slot (K - L) mod LK, and the new cost[i] replaces the oldest one, slot K.
    // The steps have no branches: a lane whose line is done (it >= m) keeps
    // stepping on bytes at or just before its line start, but stores into its
    // sink byte and keeps its costs, so that the group is one block the
    // scheduler can interleave.  Escapes are collected in *escm.
    // GL: the bytes a step group reads two places back, [lo, lo + LK), loaded one
    // group ahead (byte lo + j in bits 8j of w[j / 8])
    struct Win {
        uint64_t w[LK / 8];
    };
    __device__ __forceinline__ Win load_win(const uint8_t* buf, int32_t lo) {
        const uintptr_t ad = (uintptr_t)(buf + lo);
        const uint64_t* a = (const uint64_t*)(ad & ~(uintptr_t)7);
        const uint32_t sh = 8u * (uint32_t)(ad & 7);
        uint64_t v[LK / 8 + 1];
#pragma unroll
        for (int j = 0; j <= LK / 8; j++) v[j] = a[j];
        Win r;
#pragma unroll
        for (int j = 0; j < LK / 8; j++) r.w[j] = sh ? (v[j] >> sh) | (v[j + 1] << (64 - sh)) : v[j];
        return r;
    }

    // GL: a forward reader of one lane's bytes in global memory, 16 bytes at a
    // time with the next 16 already loaded, so that a walk whose next address
    // depends on the byte just read does not wait for memory at every byte.
    struct TokWin {
        uintptr_t wa = 0;  // address of the 16 bytes in cw
        uint4 cw, nw;
        __device__ __forceinline__ void init(const uint8_t* p) {
            wa = (uintptr_t)p & ~(uintptr_t)15;
            cw = *(const uint4*)wa;
            nw = *(const uint4*)(wa + 16);
        }
        __device__ __forceinline__ uint32_t get(const uint8_t* p) {
            const uintptr_t ad = (uintptr_t)p;
            while (ad >= wa + 16) {
                cw = nw;
                wa += 16;
                nw = *(const uint4*)(wa + 16);
            }
            const uint32_t i = (uint32_t)(ad - wa);
            // values, not fields: a choice between fields would keep the window in memory
            const uint32_t x = cw.x, y = cw.y, z = cw.z, u = cw.w;
            const uint32_t w = i < 8 ? (i < 4 ? x : y) : (i < 12 ? z : u);
            return (w >> (8 * (i & 3))) & 0xFFu;
        }
    };

    // GL: the group's code bytes are collected in cw (byte j of the group, from
    // its lowest position, in byte j % 4 of cw[j / 4]) and stored at once.
    template <int K>
    __device__ __forceinline__ void parse_steps(ParseState& ps, uint8_t* buf, uint32_t base, uint32_t m,
                                                uint32_t top, int32_t P, uint8_t* sink, uint32_t Cs,
                                                uint32_t* escm, const Win& win, uint32_t* cw) {
        if constexpr (K < LK) {
            const uint32_t it = base + K;
            const bool act = it < m;
            {
                const int32_t pos = (int32_t)top - (int32_t)it;
                const uint32_t s = ps.s;
                // the next state and the byte two places back are independent of the DP below
                const uint32_t sn = TRANS[__umul24(s, Cs) + ps.coln];
                uint32_t cnn;
                if constexpr (GL) {
                    cnn = (uint32_t)(win.w[(LK - 1 - K) / 8] >> (8 * ((LK - 1 - K) % 8))) & 0xFFu;
                } else {
                    cnn = buf[max(pos, P) - 2];  // may read just before the line: any byte will do
                }
                const uint32_t colnn = COL[cnn];
                // the state's key bits for L = 1..LK, one signed byte each (-1: no pattern),
                // in one 8- or 16-byte LDS read; sign-extended, each ORs into a cost key
                uint32_t kw[LK / 4];
                if constexpr (LK == 8) {
                    const uint2 v = *(const uint2*)(OUTK + s * LK);
                    kw[0] = v.x;
                    kw[1] = v.y;
                } else {
                    const uint4 v = *(const uint4*)(OUTK + s * LK);
                    kw[0] = v.x;
                    kw[1] = v.y;
                    kw[2] = v.z;
                    kw[3] = v.w;
                }
                uint32_t Kmin = ps.V[(K + LK - 1) % LK] + 63u;  // escape: cost[i+1] + 2, low bits 31
#pragma unroll
                for (int q = 0; q < LK; q += 2) {
                    const uint32_t e0 = (uint32_t)(int32_t)(int8_t)(kw[q >> 2] >> (8 * (q & 3)));
                    const uint32_t e1 = (uint32_t)(int32_t)(int8_t)(kw[(q + 1) >> 2] >> (8 * ((q + 1) & 3)));
                    Kmin = min(Kmin, min(ps.V[(K + 2 * LK - 1 - q) % LK] | e0, ps.V[(K + 2 * LK - 2 - q) % LK] | e1));
                }
                const uint32_t ch = 31u - (Kmin & 31u);
                // the byte to store, always one load: the code of length ch, the
                // one-byte code of c, or (escape) c itself
                const uint32_t tb = (ch >= 2) ? off_code + s * LK - 1 : (ch == 1) ? off_code1 : L.ident;
                const uint32_t t = smem[tb + ((ch >= 2) ? ch : ps.c)];
                if constexpr (GL) {
                    cw[(LK - 1 - K) / 4] |= t << (8 * ((LK - 1 - K) % 4));
                } else {
                    *(act ? buf + pos : sink) = (uint8_t)t;
                }
                *escm |= ((act && ch == 0) ? 1u : 0u) << K;
                ps.V[K] = act ? (Kmin | 31u) + 1u : ps.V[K];
                ps.s = sn;
                ps.c = ps.cn;
                ps.cn = cnn;
                ps.coln = colnn;
            }
            parse_steps<K + 1>(ps, buf, base, m, top, P, sink, Cs, escm, win, cw);
        }
    }

    // Bytes [lo, hi) (0 <= lo, hi <= 4) of a dword as a mask.
    __device__ static inline uint32_t byte_mask(int32_t lo, int32_t hi) {
        lo = max(lo, 0);
        hi = min(hi, 4);
        if (hi <= lo) return 0u;
        const uint32_t up = hi == 4 ? 0xFFFFFFFFu : ((1u << (8 * hi)) - 1u);
        return up & ~((1u << (8 * lo)) - 1u);
    }

    // Binned mode: copy lines [b0, b1) of the tile to RAW at their packed
    // offsets OFF - OFF[b0].  Each thread fills 16-byte pieces of RAW; the line
    // of a piece comes from a search of OFF, and each line the piece overlaps
    // adds its bytes: from two aligned 16-byte loads shifted into place, or byte
    // by byte where those loads would leave the input.  A bad line is a lone
    // newline; a virtual final newline is not in memory.
    __device__ __forceinline__ void load_gather(uint32_t b0, uint32_t b1, uint8_t* raw) {
        const uint64_t* off = OFF();
        const uint64_t* abs = ABS();
        const uint32_t lo = (uint32_t)off[b0], n = (uint32_t)off[b1] - lo;
        const uintptr_t ib = (uintptr_t)A.in, ie = ib + A.in_bytes;
        for (uint32_t r0 = threadIdx.x * 16; r0 < n; r0 += kWG * 16) {
            uint32_t l = b0, h = b1;
            while (h - l > 1) {
                const uint32_t mid = (l + h) >> 1;
                if ((uint32_t)off[mid] - lo <= r0) l = mid;
                else h = mid;
            }
            uint32_t q = l;
            uint32_t qs = (uint32_t)off[q] - lo, qe = (uint32_t)off[q + 1] - lo;
            const uint32_t pe = min(r0 + 16, n);  // end of the piece's bytes
            uint32_t w[4] = {0, 0, 0, 0};
            while (true) {
                // bytes [s0, s1) of the piece come from line q
                const uint32_t s0 = max(qs, r0), s1 = min(qe, pe);
                const uint64_t a = abs[q];
                const bool bad = (a & kAbsBad) != 0;
                const uint64_t src = a & ~kAbsBad;
                const uintptr_t sa = ib + src + (s0 - qs);
                const uintptr_t c0 = sa & ~(uintptr_t)15;
                if (!bad && c0 >= ib && c0 + 32 <= ie) {
                    // (the newline of such a line is in memory: a virtual one would lie past ie)
                    const uint4 x = *(const uint4*)c0, y = *(const uint4*)(c0 + 16);
                    // piece byte k is byte k + e of 16 zero bytes, then x, then y
                    const uint32_t e = (uint32_t)(sa - c0) + 16u - (s0 - r0);
                    const uint32_t z[12] = {0u, 0u, 0u, 0u, x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
                    const uint32_t qd = e >> 2, rb = e & 3u;
                    uint32_t d[5];
#pragma unroll
                    for (int j = 0; j < 5; j++) {
                        uint32_t v = 0;
#pragma unroll
                        for (int c = 0; c < 8; c++) v = qd == (uint32_t)c ? z[c + j] : v;
                        d[j] = v;
                    }
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const uint32_t m = byte_mask((int32_t)(s0 - r0) - 4 * j, (int32_t)(s1 - r0) - 4 * j);
                        w[j] |= __builtin_amdgcn_alignbyte(d[j + 1], d[j], rb) & m;
                    }
                } else {
                    const bool vnl = !bad && src + (qe - qs) == A.in_bytes + 1;
                    for (uint32_t r = s0; r < s1; r++) {
                        uint32_t v = 0;
                        if (r + 1 == qe && (bad || vnl)) v = '\n';
                        else if (!bad) v = A.in[src + (r - qs)];
                        w[(r - r0) >> 2] |= v << (8 * ((r - r0) & 3));
                    }
                }
                if (qe >= pe) break;
                q++;
                qs = qe;
                qe = (uint32_t)off[q + 1] - lo;
            }
            if (r0 + 16 <= n) {
                *(uint4*)(raw + r0) = make_uint4(w[0], w[1], w[2], w[3]);
            } else {
                for (uint32_t k = 0; r0 + k < n; k++) raw[r0 + k] = (uint8_t)(w[k >> 2] >> (8 * (k & 3)));
            }
        }
    }

    // Process lines [b0, ...) of the tile as one batch: load, ring IDs, expand,
    // parse.  Fills COST for the batch lines and returns b1.  The per-lane
    // state needed for emission is left in `st`.
    __device__ __forceinline__ uint32_t batch(uint64_t k0, uint32_t nl, uint32_t b0, bool regular, LineState& st) {
        uint32_t* misc = MISC();
        uint64_t* off = OFF();
        uint8_t* raw = RAW();
        uint8_t* pre = PRE();
        uint16_t* lens = LENS();
        uint16_t* perm = PERM();
        const uint32_t tid = threadIdx.x;
        const bool prep = (A.flags & ZS_F_PREPROCESS) != 0;
        // ---- extent of the batch
        if (tid == 0) misc[0] = nl;
        bar();
        {
            const uint32_t j = b0 + tid;
            if (j < nl && j > b0) {
                const bool stop = !regular || (off[j + 1] - off[b0]) + 16 > (uint64_t)kRawCap;
                if (stop) atomicMin(&misc[0], j);
            }
        }
        bar();
        uint32_t b1 = misc[0];
        bar();
        bool marked_lane = false;
        bool gen_lane = false;  // the line's markers are ring_general's (GL expansion)
        uint32_t ext = 0;  // bytes of RAW or PRE the batch uses (GL: the escape bits cleared)
        while (true) {
            const uint32_t nb = b1 - b0;
            if constexpr (GL) {
                // the label bytes of the ring tables start at zero at every attempt (the
                // dictionary's LDS, free until the parse; the barriers below order this)
                for (uint32_t k = tid; k < (uint32_t)kLabels * kWG / 16; k += kWG)
                    ((uint4*)(smem + L.ring))[k] = make_uint4(0, 0, 0, 0);
            }
            // ---- load
            const uint32_t fe0 = frame_error(k0, b0);
            const uint64_t lo = off[b0];
            uint32_t base_off = 0;
            if (A.ids) {
                load_gather(b0, b1, raw);
            } else {
                uint64_t hi = off[b1];
                if (hi > A.in_bytes) hi = A.in_bytes;
                const uintptr_t a0 = ((uintptr_t)(A.in + lo)) & ~(uintptr_t)15;
                base_off = (uint32_t)((uintptr_t)(A.in + lo) - a0);
                if (fe0 == 0) load_range(A.in, A.in_bytes, lo, hi, a0, raw);
                bar();
                if (tid == 0 && fe0 == 0 && off[b1] == A.in_bytes + 1)
                    raw[(uint32_t)(off[b1] - 1 - lo) + base_off] = '\n';
            }
            bar();
            // ---- framing per line, lengths for the rank order
            if (tid < nb) {
                const uint32_t j = b0 + tid;
                uint32_t fe = frame_error(k0, j);
                uint32_t len = 0;
                if (fe == 0) {
                    len = (uint32_t)(off[j + 1] - off[j] - 1);
                    if (raw[(uint32_t)(off[j] - lo) + base_off + len] != '\n') fe = kErrInval;
                }
                if (fe) note_error(A.ws, line_id(k0, j), fe);
                lens[tid] = fe ? (uint16_t)kBadLine : (uint16_t)len;
            }
            bar();
            // ---- rank lines by length (buckets of 8 bytes) so that a wave holds lines of
            //      similar length; the order inside a bucket does not affect any result
            {
                uint32_t* cnt = ESC();  // scratch until the escape bits are cleared
                if (tid < 64) cnt[tid] = 0;
                bar();
                uint32_t bk = 0, within = 0;
                if (tid < nb) {
                    const uint32_t lj = lens[tid];
                    bk = (lj & kBadLine) ? 0u : min(lj >> 3, 31u);
                    within = atomicAdd(&cnt[bk], 1u);
                }
                bar();
                if (tid < 32) {
                    const uint32_t v = cnt[tid];
                    uint32_t inc = v;
#pragma unroll
                    for (int d = 1; d < 32; d <<= 1) {
                        const uint32_t u = __shfl_up(inc, d, 64);
                        if ((int)tid >= d) inc += u;
                    }
                    cnt[32 + tid] = inc - v;
                }
                bar();
                if (tid < nb) perm[cnt[32 + bk] + within] = (uint16_t)tid;
            }
            bar();
            // wave w takes the ((w + rot) mod 4)-th quarter of the length order:
            // the wave with the longest lines moves from tile to tile, so that
            // it does not sit on the same SIMD in every workgroup of the CU
            const uint32_t rq = (tid + 64u * (blockIdx.x + ((uint32_t)k0 >> 8))) & (kWG - 1);
            st.in = rq < nb;
            st.j = st.in ? perm[rq] : 0u;
            const uint32_t lj = st.in ? lens[st.j] : 0u;
            st.bad = st.in && (lj & kBadLine);
            st.len = (st.in && !st.bad) ? lj : 0u;
            st.R = st.in ? (uint32_t)(off[b0 + st.j] - lo) + base_off : 0u;
            st.m = 0;
            // ---- ring IDs (Sec. IV-A)
            bool overflow = false, malformed = false, run_rings = false;
            int delta = 0;
            const uint32_t line = b0 + st.j;
            // the label list sits in PRE under the line (PRE is written only after the ring pass)
            uint16_t* list = (uint16_t*)pre + ((st.R + 1) >> 1);
            uint32_t* list32 = (uint32_t*)(pre + ((st.R + 15) & ~15u));
            uint32_t nlab = 0;
            if (st.in && !st.bad) {
                bool corrupt, over, pct;
                if constexpr (GL) {
                    const uint32_t le = (st.R + st.len) & ~15u, ls = (st.R + 15) & ~15u;
                    scan_labels(raw, st.R, st.len, list32, le > ls ? (le - ls) / 4 : 0u, &nlab, &corrupt, &malformed,
                                &over, &pct);
                } else {
                    scan_labels(raw, st.R, st.len, list, st.len >> 1, &nlab, &corrupt, &malformed, &over, &pct);
                }
                if (corrupt) {
                    st.bad = true;
                    note_error(A.ws, line_id(k0, line), kErrCorrupt);
                } else if (prep && !malformed) {
                    if (over) overflow = true;
                    else run_rings = true;
                }
            }
            // GL: the scan's entry queues share LDS with other lanes' ring slots
            if constexpr (GL) bar();
            // the label loop runs to the wave's longest list (all lanes take part in the max)
            uint32_t maxlab = run_rings ? nlab : 0u;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) maxlab = max(maxlab, (uint32_t)__shfl_xor((int)maxlab, d, 64));
            bool marked = false;
            constexpr bool post = MODE == kModePost;
            if (run_rings) {
                bool ok;
                if constexpr (GL) {
                    // long lines hold many rings open at once: the label tables
                    static_assert(!GL || MODE == kModeCompress, "the global-memory layout only compresses");
                    ok = ring_table(raw, st.R, list32, nlab, maxlab, &delta, &overflow, &marked);
                } else {
                    // a table of 4 slots first (more rings than that are rarely open at
                    // once), 8 for the lines it cannot hold
                    ok = ring_fast<kSlotsFirst, post>(raw, st.R, list, nlab, maxlab, &delta, &overflow, &marked);
                    if (overflow) {
                        restore_line(raw, st.R, line_src(line), st.len);
                        overflow = false;
                        ok = ring_fast<kSlots, post>(raw, st.R, list, nlab, maxlab, &delta, &overflow, &marked);
                    }
                }
                if (!ok && !overflow) {
                    malformed = true;
                    restore_line(raw, st.R, line_src(line), st.len);
                }
            }
            if (overflow) {
                restore_line(raw, st.R, line_src(line), st.len);
                uint16_t* open = (uint16_t*)(A.gen + ((uint64_t)blockIdx.x * kWG + tid) * kGenLane);
                if (!ring_general<post>(raw, st.R, st.len, open, open + 100, &delta)) {
                    malformed = true;
                    restore_line(raw, st.R, line_src(line), st.len);
                } else {
                    marked = true;
                    gen_lane = true;
                }
            }
            if (malformed) marked = gen_lane = false;  // restored: the raw bytes are the line
            marked_lane = marked;
            if (st.in && !st.bad) st.m = (prep && !malformed) ? (uint32_t)((int)st.len + delta) : st.len;
            // ---- pack the pre-processed lines (in lane order)
            // GL: each line ends on a 16-byte boundary, its padding in front of it
            uint32_t total;
            const uint32_t mm = st.in ? st.m : 0u;
            const uint32_t slot = GL ? (mm + 15u) & ~15u : mm;
            st.P = block_excl_scan(slot, misc + 4, &total) + (slot - mm);
            if constexpr (GL) ext = max(total, (uint32_t)(off[b1] - lo) + base_off);
            if (total <= (uint32_t)kPreCap) break;
            // rare: growth made PRE overflow; redo with fewer lines
            b1 = b0 + max(1u, nb / 2);
            bar();
        }
        // ---- expand markers into PRE (only when some line changed length; GL:
        //      always, into the aligned layout)
        if constexpr (GL) st.simple = false;
        else st.simple = bar_or(st.in && !st.bad && marked_lane) == 0;
        if (st.simple) st.P = st.R;
        if (!st.simple && st.in && !st.bad && st.m) {
            const uint32_t end = st.R + st.len;
            if constexpr (GL) {
                // 16-byte loads one chunk ahead.  The bytes go through a 32-byte ring of
                // this lane in LDS (byte s of the ring in byte s % 4 of row s / 4, rows
                // kWG dwords apart) and out as aligned 16-byte blocks, at most one per
                // input word; the first block starts in the line's padding and the
                // last one ends with the line.
                uint8_t* ring = smem + L.ring + 4 * threadIdx.x;
                uint32_t wpos = st.P, fb = st.P & ~15u;
                const uint32_t c0 = st.R & ~15u;
                uint4 nx = *(const uint4*)(raw + c0);
                // markers: ring_general's drop a byte (kSkip) or carry an ID below 100;
                // the label tables' carry an ID below 32, with 0x40 when the two digits
                // of a '%' label follow (dropped here)
                const uint32_t idm = gen_lane ? 0x7Fu : 0x3Fu;
                uint32_t sk = 0;  // digits still to drop
                for (uint32_t c = c0; c < end; c += 16) {
                    const uint4 cu = nx;
                    nx = *(const uint4*)(raw + c + 16);  // at most 31 bytes past the line: in the buffer
                    const uint32_t wd[4] = {cu.x, cu.y, cu.z, cu.w};
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        const uint32_t x = c + k;
                        const uint32_t b = (wd[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                        const bool mark = b >= kIdMark;
                        const uint32_t id = b & idm;
                        const bool inr = x >= st.R && x < end;
                        const bool in = inr && b != kSkip && sk == 0;
                        if (inr) sk = sk ? sk - 1 : ((!gen_lane && mark && (b & 0x40u)) ? 2u : 0u);
                        const bool three = mark && id >= 10;
                        const uint32_t b0 = three ? '%' : (mark ? '0' + id : b);
                        if (in) {
                            const uint32_t sl = wpos & 31u;
                            ring[(sl >> 2) * (kWG * 4) + (sl & 3u)] = (uint8_t)b0;
                            wpos++;
                            if (three) {
                                const uint32_t s1 = wpos & 31u, s2 = (wpos + 1) & 31u;
                                ring[(s1 >> 2) * (kWG * 4) + (s1 & 3u)] = (uint8_t)('0' + id / 10);
                                ring[(s2 >> 2) * (kWG * 4) + (s2 & 3u)] = (uint8_t)('0' + id % 10);
                                wpos += 2;
                            }
                        }
                        if ((k & 3) == 3 && wpos - fb >= 16) {
                            const uint32_t* rw = (const uint32_t*)(ring + ((fb & 16u) >> 2) * (kWG * 4));
                            *(uint4*)(pre + fb) = make_uint4(rw[0], rw[kWG], rw[2 * kWG], rw[3 * kWG]);
                            fb += 16;
                        }
                    }
                }
                while (fb < wpos) {  // wpos = P + m, a 16-byte boundary
                    const uint32_t* rw = (const uint32_t*)(ring + ((fb & 16u) >> 2) * (kWG * 4));
                    *(uint4*)(pre + fb) = make_uint4(rw[0], rw[kWG], rw[2 * kWG], rw[3 * kWG]);
                    fb += 16;
                }
            } else {
                uint32_t wpos = st.P;
                for (uint32_t w = st.R & ~3u; w < end; w += 4) {
                    const uint32_t word = *(const uint32_t*)(raw + w);
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const uint32_t x = w + k;
                        if (x >= st.R && x < end) {
                            const uint32_t c = (word >> (8 * k)) & 0xFFu;
                            if (c < kSkip) {
                                pre[wpos++] = (uint8_t)c;
                            } else if (c >= kIdMark) {
                                const uint32_t id = c & 0x7F;
                                if (id < 10) {
                                    pre[wpos++] = (uint8_t)('0' + id);
                                } else {
                                    pre[wpos++] = '%';
                                    pre[wpos++] = (uint8_t)('0' + id / 10);
                                    pre[wpos++] = (uint8_t)('0' + id % 10);
                                }
                            }
                        }
                    }
                }
            }
        }
        {
            uint32_t* esc = ESC();
            const uint32_t words = GL ? min((ext + 32u) / 32u, (uint32_t)kPreCap / 32u) : (uint32_t)kPreCap / 32u;
            for (uint32_t k = tid; k < words; k += kWG) esc[k] = 0;
        }
        if constexpr (GL) {
            // the dictionary back into its LDS, once every lane is past the expansion
            bar();
            for (uint32_t k = tid; k < L.tab_bytes / 16; k += kWG) ((uint4*)smem)[k] = ((const uint4*)A.tables)[k];
        }
        bar();
        // ---- parse (backward): automaton + (min,+) window over the next LK costs
        uint32_t cost = 0;
        bool esc_any = false;
        constexpr bool preonly = MODE != kModeCompress;
        if constexpr (preonly) {
            cost = (st.in && !st.bad) ? st.m : 0u;  // the output line is the relabelled line
        } else {
            uint8_t* buf = st.simple ? raw : pre;
            const uint32_t m = (st.in && !st.bad) ? st.m : 0u;
            uint32_t mx = m;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
            ParseState ps;
#pragma unroll
            for (int k = 0; k < LK; k++) ps.V[k] = 0xFFFFFFFFu;
            ps.V[LK - 1] = 32u;  // cost[m] = 0, as (cost + 1) << 5
            const uint32_t top = st.P + m - 1;  // position of the last byte (unused when m == 0)
            ps.c = buf[(int)top];
            ps.s = TRANS[COL[ps.c]];
            ps.cn = buf[(int)top - 1];
            ps.coln = COL[ps.cn];
            uint8_t* sink = smem + L.sink + threadIdx.x;
            const uint32_t Cs = __builtin_amdgcn_readfirstlane(C);
            // GL: the group's bytes two places back come from a window loaded one group
            // ahead (a lane whose line has ended reads any in-bounds bytes)
            Win nwin;
            if constexpr (GL) nwin = load_win(buf, max((int32_t)top - LK - 1, (int32_t)st.P - LK - 2));
            for (uint32_t base = 0; base < mx; base += LK) {
                uint32_t escm = 0;
                Win win;
                if constexpr (GL) {
                    win = nwin;
                    nwin = load_win(buf, max((int32_t)top - (int32_t)(base + LK) - LK - 1, (int32_t)st.P - LK - 2));
                }
                uint32_t cw[LK / 4];
#pragma unroll
                for (int k = 0; k < LK / 4; k++) cw[k] = 0;
                parse_steps<0>(ps, buf, base, m, top, (int32_t)st.P, sink, Cs, &escm, win, cw);
                if constexpr (GL) {
                    // the group's bytes end on an LK-aligned position (lines end on 16-byte
                    // boundaries); bytes before the line's start fall in its padding
                    if (base < m) {
                        uint8_t* g = buf + (top - base - (LK - 1));
                        if constexpr (LK == 8) *(uint2*)g = make_uint2(cw[0], cw[1]);
                        else *(uint4*)g = make_uint4(cw[0], cw[1], cw[2], cw[3]);
                    }
                }
                esc_any |= escm != 0;
                for (; escm; escm &= escm - 1) {  // rare: bytes with no code of their own
                    const uint32_t pos = top - (base + (uint32_t)__builtin_ctz(escm));
                    atomicOr(&ESC()[pos >> 5], 1u << (pos & 31));
                }
            }
            if (m) {
                const uint32_t last = (m - 1) & (LK - 1);
                uint32_t v = 0;
#pragma unroll
                for (int k = 0; k < LK; k++) v = ((uint32_t)k == last) ? ps.V[k] : v;
                cost = (v >> 5) - 1u;
            }
        }
        // a compressed line longer than the decoder takes is bad, like a raw line
        // longer than ZS_MAX_LINE (only renumbering that lengthens a line can get there)
        if (!preonly && st.in && !st.bad && cost > ZS_MAX_CLINE) {
            st.bad = true;
            note_error(A.ws, line_id(k0, b0 + st.j), kErrInval);
        }
        if (st.in) COST()[b0 + st.j] = st.bad ? 0u : cost;
        st.esc = bar_or(esc_any) != 0;
        return b1;
    }

    // Emit the lines of the batch held in LDS into the output, one stage window
    // at a time.  gbase: global output offset of the tile.
    // rel: write the batch at tile-relative offsets from stage byte 0 and leave it
    // there (one window; the caller copies it out later).
    __device__ __forceinline__ void emit(uint32_t b0, uint32_t b1, const LineState& st, uint64_t gbase, bool rel = false) {
        uint8_t* stage = st.simple ? PRE() : RAW();        // the buffer not holding tokens
        const uint8_t* pre = st.simple ? RAW() : PRE();
        const uint32_t* esc = ESC();
        const uint64_t gb0 = gbase + EOFF()[b0];
        const uint64_t gb1 = gbase + EOFF()[b1 - 1] + COST()[b1 - 1] + 1;
        const uint32_t m = (st.in && !st.bad) ? st.m : 0u;
        uint32_t ic = 0;
        bool nl_done = !st.in;
        uint64_t oc = st.in ? gbase + EOFF()[b0 + st.j] : 0;
        if (gb1 - gb0 <= (uint64_t)(kRawCap - 16)) {
            // the batch's output fits one window: each lane appends its line
            // (codes, escapes, newline) with dword stores
            const uintptr_t a0 = rel ? 0 : (((uintptr_t)(A.out + gb0)) & ~(uintptr_t)15);
            const uintptr_t sbase = rel ? 0 : (uintptr_t)A.out - a0;
            if constexpr (GL && MODE == kModeCompress) {
                if (st.in) {
                    // the bytes go through a 32-byte ring of this lane in LDS (after the
                    // dictionary) and out as aligned 16-byte blocks, at most one every
                    // four codes; blocks shared with the neighbouring lines byte by byte
                    uint8_t* rg = smem + L.eri + 4 * threadIdx.x;
                    const uint32_t s0 = (uint32_t)(sbase + oc);
                    uint32_t wp = s0, fb = s0 & ~15u, n = 0;
                    auto putb = [&](uint32_t b) __attribute__((always_inline)) {
                        const uint32_t sl = wp & 31u;
                        rg[(sl >> 2) * (kWG * 4) + (sl & 3u)] = (uint8_t)b;
                        wp++;
                    };
                    auto flush = [&](uint32_t hi) __attribute__((always_inline)) {
                        const uint8_t* rb = rg + ((fb & 16u) >> 2) * (kWG * 4);
                        if (fb >= s0 && hi == fb + 16) {
                            const uint32_t* rw = (const uint32_t*)rb;
                            *(uint4*)(stage + fb) = make_uint4(rw[0], rw[kWG], rw[2 * kWG], rw[3 * kWG]);
                        } else {
                            for (uint32_t x = max(fb, s0); x < hi; x++)
                                stage[x] = rb[((x & 15u) >> 2) * (kWG * 4) + (x & 3u)];
                        }
                        fb += 16;
                    };
                    TokWin tw;
                    tw.init(pre + st.P);
                    uint32_t ew = 0, ewi = ~0u;  // the escape-bit word last read
                    while (ic < m) {
                        const uint32_t pos = st.P + ic;
                        const uint32_t t = tw.get(pre + pos);
                        bool e = false;
                        if (st.esc) {
                            if ((pos >> 5) != ewi) {
                                ewi = pos >> 5;
                                ew = esc[ewi];
                            }
                            e = ((ew >> (pos & 31)) & 1u) != 0;
                        }
                        if (e) {
                            putb(0x20);
                            putb(t);
                            ic += 1;
                        } else {
                            putb(t);
                            ic += LENT[t];
                        }
                        if ((++n & 3u) == 0 && wp - fb >= 16) flush(fb + 16);
                    }
                    putb('\n');
                    while (fb < wp) flush(min(fb + 16, wp));
                }
            } else if constexpr (MODE != kModeCompress) {
                // relabelling only: the line's bytes and its newline
                if (st.in) {
                    StageWriter wr;
                    wr.begin(stage, (uint32_t)(sbase + oc));
                    for (; ic < m; ic++) wr.add(pre[st.P + ic], 1);
                    wr.add('\n', 1);
                    wr.finish();
                }
            } else if (st.in && !st.esc) {
                // one byte per code: a 32-bit accumulator, dword stores, bytes
                // only in the dwords shared with the neighbouring lines
                uint32_t* st32 = (uint32_t*)stage;
                const uint32_t s0 = (uint32_t)(sbase + oc), lead = s0 & 3u, a0 = s0 >> 2;
                uint32_t a = a0, p = lead, acc = 0;
                auto put = [&]() {
                    if (a == a0 && lead) {
                        for (uint32_t j = lead; j < 4; j++) stage[4 * a + j] = (uint8_t)(acc >> (8 * j));
                    } else {
                        st32[a] = acc;
                    }
                    a++;
                    p = 0;
                    acc = 0;
                };
                while (ic < m) {
                    const uint32_t t = pre[st.P + ic];
                    acc |= t << (8 * p);
                    ic += LENT[t];
                    if (++p == 4) put();
                }
                acc |= (uint32_t)'\n' << (8 * p);
                if (++p == 4) put();
                for (uint32_t j = (a == a0 ? lead : 0u); j < p; j++) stage[4 * a + j] = (uint8_t)(acc >> (8 * j));
            } else if (st.in) {
                StageWriter wr;
                wr.begin(stage, (uint32_t)(sbase + oc));
                while (ic < m) {
                    const uint32_t pos = st.P + ic;
                    const uint32_t t = pre[pos];
                    const uint32_t eb = esc[pos >> 5];
                    if ((eb >> (pos & 31)) & 1u) {
                        wr.add(0x20u | (t << 8), 2);
                        ic += 1;
                    } else {
                        wr.add(t, 1);
                        ic += LENT[t];
                    }
                }
                wr.add('\n', 1);
                wr.finish();
            }
            bar();
            if (!rel) flush_stage(A.out, gb0, gb1, a0, stage);
            bar();
            return;
        }
        uint64_t wlo = gb0;
        while (wlo < gb1) {
            uint64_t whi = wlo + (uint64_t)(min(kRawCap, kPreCap) - 16);
            if (whi > gb1) whi = gb1;
            const uintptr_t a0 = rel ? 0 : (((uintptr_t)(A.out + wlo)) & ~(uintptr_t)15);
            const uintptr_t sbase = rel ? 0 : (uintptr_t)A.out - a0;  // stage index of offset g = sbase + g
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
                        adv = MODE != kModeCompress ? 1u : LENT[t];
                    }
                } else {
                    b[0] = '\n';
                    tl = 1;
                    adv = 0;
                }
                for (uint32_t k = 0; k < tl; k++) {
                    const uint64_t g = oc + k;
                    if (g >= wlo && g < whi) stage[sbase + g] = (uint8_t)b[k];
                }
                if (oc + tl > whi) break;
                oc += tl;
                if (ic < m) ic += adv;
                else nl_done = true;
            }
            bar();
            if (!rel) flush_stage(A.out, wlo, whi, a0, stage);
            bar();
            wlo = whi;
        }
    }

    // Tiles are processed in ticket order.  A tile whose output fits one stage
    // window publishes its size as soon as it is parsed, parks its bytes in this
    // workgroup's global slot and is placed one tile later, when its
    // predecessors have published: no workgroup waits on a slower neighbour.
    // Other tiles (several batches, or large output) are placed at once.
    __device__ __forceinline__ void run() {
        uint32_t* misc = MISC();
        uint64_t* off = OFF();
        const uint32_t tid = threadIdx.x;
        uint8_t* slot = A.slots + (uint64_t)blockIdx.x * kSlotBytes;
        bool pend = false;
        uint32_t pt = 0, pnl = 0, ptotal = 0, prel = 0;
        uint64_t pk0 = 0;
        while (true) {
            uint32_t t, nl = 0;
            uint64_t k0 = 0;
            bool have;
            if (A.ids) {
                // binned mode: this launch's tiles are [first_tile[bin_lo], first_tile[bin_hi])
                if (tid == 0) misc[2] = atomicAdd(A.ticket, 1u);
                bar();
                t = A.plan->first_tile[A.bin_lo] + misc[2];
                bar();
                have = t < A.plan->first_tile[A.bin_hi];
                if (have) {
                    uint32_t b = A.bin_lo;
                    while (t >= A.plan->first_tile[b + 1]) b++;
                    const uint32_t lpt = A.plan->lpt[b];
                    k0 = A.plan->start[b] + (uint64_t)(t - A.plan->first_tile[b]) * lpt;
                    nl = (uint32_t)min((uint64_t)lpt, A.plan->start[b] + A.plan->count[b] - k0);
                }
            } else {
                t = claim_tile(A.ws, &misc[2]);
                have = t < A.ntiles;
                if (have) {
                    k0 = (uint64_t)t * kCL;
                    nl = (uint32_t)min((uint64_t)kCL, A.n - k0);
                }
            }
            LineState st;
            st.simple = true;
            st.esc = true;
            st.in = false;
            st.bad = false;
            uint32_t nb = 0, total = 0, e = 0, mylen = 0;
            bool regular = true;
            if (have) {
                if (A.ids) {
                    // packed offsets of the gathered lines; a bad line takes one byte
                    uint64_t a = 0;
                    uint32_t sz = 0;
                    if (tid < nl) {
                        const uint64_t id = A.ids[k0 + tid];
                        a = A.in_off[id];
                        const uint64_t b = A.in_off[id + 1];
                        bool bad = b <= a || b > A.in_bytes + 1 || b - a - 1 > ZS_MAX_LINE ||
                                   (b == A.in_bytes + 1 && id + 1 != A.n);
                        sz = bad ? 1u : (uint32_t)(b - a);
                        if (bad) a |= kAbsBad;
                        ABS()[tid] = a;
                    }
                    uint32_t tot;
                    const uint32_t ex = block_excl_scan(sz, misc + 4, &tot);
                    if (tid < nl) off[tid] = ex;
                    if (tid == 0) off[nl] = tot;
                } else {
                    for (uint32_t j = tid; j <= nl; j += kWG) off[j] = A.in_off[k0 + j];
                }
                if (tid < kCL) COST()[tid] = 0;
                bar();
                regular = A.ids != nullptr || bar_and(tid >= nl || frame_error(k0, tid) == 0) != 0;
                // sweep 1: parse every batch, sizes into COST
                uint32_t b0 = 0;
                while (b0 < nl) {
                    b0 = batch(k0, nl, b0, regular, st);
                    nb++;
                }
                mylen = tid < nl ? COST()[tid] + 1 : 0u;
                e = block_excl_scan(mylen, misc + 4, &total);
                if (tid < nl) EOFF()[tid] = e;
                if (tid == 0 && !A.ids) publish_aggregate(A.status, t, total);
            }
            uint8_t* stage = st.simple ? PRE() : RAW();  // the buffer not holding this tile's tokens
            // place the pending tile
            if (pend) {
                if (tid < 64) {
                    const uint64_t ex = lookback_walk(A.status, pt, ptotal);
                    if (tid == 0) ((uint64_t*)misc)[6] = ex;
                }
                bar();
                const uint64_t pbase = ((uint64_t*)misc)[6];
                if (tid < pnl) A.out_off[pk0 + tid + 1] = pbase + prel;
                if (A.out) {
                    if (pbase + ptotal <= A.out_cap) {
                        // each thread reads back only the slot chunks it wrote (a global
                        // store of another wave need not be visible after a barrier),
                        // into the free LDS buffer; the shifted copy then reads LDS
                        for (uint32_t c = tid; c < (ptotal + 15) / 16; c += kWG)
                            ((uint4*)stage)[c] = ((const uint4*)slot)[c];
                        bar();
                        copy_slot_direct(A.out, stage, ptotal, pbase);
                    } else if (tid == 0) {
                        atomicOr(&A.ws->enospc, 1u);
                    }
                }
                pend = false;
                bar();
            }
            if (!have) break;
            if (t == 0 && tid == 0 && !A.ids) A.out_off[0] = 0;
            // Binned (gather) launches place every tile at once: parked tiles gave
            // wrong bytes there under load, a cause not yet found.
            const bool defer = nb == 1 && total + 16 <= (uint32_t)kSlotBytes && A.ids == nullptr;
            if (defer) {
                prel = e + mylen;  // this line's end inside the tile, until the tile is placed
                if (A.out) {
                    emit(0, nl, st, 0, true);
                    for (uint32_t c = tid; c < (total + 15) / 16; c += kWG)
                        ((uint4*)slot)[c] = ((const uint4*)stage)[c];
                }
                pend = true;
                pt = t;
                pk0 = k0;
                pnl = nl;
                ptotal = total;
            } else {
                // binned: the tile's staging space comes from a bump allocator (the
                // placement pass reads each line's staging start and length, so the
                // staging order is free and no tile waits on another); a tile whose
                // output fits one stage window is emitted first, tile-relative into the
                // free buffer, and copied out afterwards
                const bool early = A.ids && A.out && nb == 1 && total + 16 <= (uint32_t)kSlotBytes;
                if (early) emit(0, nl, st, 0, true);
                if (A.ids) {
                    if (tid == 0) ((uint64_t*)misc)[6] = atomicAdd((unsigned long long*)&A.ws->alloc,
                                                                   (unsigned long long)total);
                } else if (tid < 64) {
                    const uint64_t ex = lookback_walk(A.status, t, total);
                    if (tid == 0) ((uint64_t*)misc)[6] = ex;
                }
                bar();
                const uint64_t gbase = ((uint64_t*)misc)[6];
                if (A.ids) {
                    // staging start << 16 | compressed length (at most ZS_MAX_CLINE + 1)
                    if (tid < nl) A.out_off[k0 + tid] = ((gbase + e) << 16) | mylen;
                } else if (tid < nl) {
                    A.out_off[k0 + tid + 1] = gbase + e + mylen;
                }
                const bool fits = gbase + total <= A.out_cap;
                if (A.out && !fits && tid == 0) atomicOr(&A.ws->enospc, 1u);
                if (A.out && fits) {
                    if (early) {
                        copy_slot_direct(A.out, stage, total, gbase);
                    } else if (nb == 1) {
                        emit(0, nl, st, gbase);
                    } else {
                        uint32_t b0 = 0;
                        while (b0 < nl) {
                            const uint32_t b1 = batch(k0, nl, b0, regular, st);
                            emit(b0, b1, st, gbase);
                            b0 = b1;
                        }
                    }
                }
            }
            bar();
        }
    }
};

template <int LK, int CAP, int MODE, bool GL>
__device__ __forceinline__ void compress_body(const CompressArgs& a) {
    extern __shared__ __align__(16) uint8_t smem[];
    // stage the dictionary image (up to EXP) in LDS
    {
        const uint4* src = (const uint4*)a.tables;
        uint4* dst = (uint4*)smem;
        for (uint32_t k = threadIdx.x; k < a.tab_bytes / 16; k += kWG) dst[k] = src[k];
        smem[compress_lds(a.tab_bytes, CAP, GL).ident + threadIdx.x] = (uint8_t)threadIdx.x;
    }
    __syncthreads();
    Compressor<LK, CAP, MODE, GL> c(a, smem);
    c.run();
}

template <int LK, int CAP, int MODE = kModeCompress>
__global__ void __launch_bounds__(kWG) compress_kernel(CompressArgs a) {
    compress_body<LK, CAP, MODE, false>(a);
}

// The global-memory layout holds little in LDS, so its occupancy is set by
// registers: kept at three waves per SIMD (at most 168 VGPRs).
template <int LK>
__global__ void __launch_bounds__(kWG, 3) compress_kernel_gl(CompressArgs a) {
    compress_body<LK, kCapGlobal, kModeCompress, true>(a);
}

// ============================================================================
// Decompression (bulk and random access)
// ============================================================================

constexpr int kDL = 256;                 // lines (or requests) per tile
constexpr int kCbCap = 8192 + 16;        // LDS bytes of compressed lines per batch
constexpr uint32_t kMaxCLine = ZS_MAX_CLINE;  // longest compressed line accepted (newline excluded)
static_assert(kMaxCLine + 1 + 15 <= (uint32_t)kCbCap, "a longest line, its newline and the lead must fit CB");
constexpr int kSeg = kWG * 16;           // bytes per decode segment
constexpr int kDStage = 16384;           // LDS output stage (a multiple of 16)

// A decompression call is one launch: tiles are taken in ticket order, sized,
// placed by a decoupled look-back and emitted.

struct DecompressLds {
    uint32_t tabs, cb, qoff, llen, bad, off, misc, stage, total;
};

__host__ __device__ inline DecompressLds decompress_lds() {
    DecompressLds L;
    uint32_t o = 0;
    L.tabs = o;   o += 64 + 256 + 256 * kExpStride;  // header, LEN, EXP
    o = align16(o);
    L.cb = o;     o += align16(kCbCap + 16);
    L.qoff = o;   o += (kDL + 1) * 4;
    L.llen = o;   o += kDL * 4;
    L.bad = o;    o += kDL;
    o = align16(o);
    L.off = o;    o += (kDL + 1) * 16;  // a and b per line
    L.misc = o;   o += 256;
    L.stage = align16(o);
    L.total = L.stage + kDStage;
    return L;
}

struct DecompressArgs {
    const uint8_t* tables;
    uint32_t off_len, off_exp;  // offsets of LEN and EXP in the table blob
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
    uint32_t tl;                // lines (requests) per tile, at most kDL
    WsHeader* ws;
    uint64_t* status;           // look-back words, one per tile
};

// misc words of the decoder (uint32 indices)
constexpr int kDmB1 = 0, kDmSlot = 2, kDmScanA = 16, kDmScanB = 24, kDmBase64 = 32;

struct Decoder {
    const DecompressArgs A;
    uint64_t r0 = 0;  // first request of the current tile
    uint8_t* smem;
    DecompressLds L;
    const uint8_t* LEN;
    const uint8_t* EXP;
    bool lmax8;  // every expansion fits 8 bytes

    __device__ Decoder(const DecompressArgs& a, uint8_t* s) : A(a), smem(s) {
        L = decompress_lds();
        LEN = smem + 64;
        EXP = smem + 64 + 256;
        lmax8 = ((const TableHeader*)smem)->lmax <= 8;
    }
    __device__ __forceinline__ uint8_t* CB() { return smem + L.cb; }
    __device__ __forceinline__ uint32_t* QOFF() { return (uint32_t*)(smem + L.qoff); }
    __device__ __forceinline__ uint32_t* LLEN() { return (uint32_t*)(smem + L.llen); }
    __device__ __forceinline__ uint8_t* BAD() { return smem + L.bad; }
    __device__ __forceinline__ uint64_t* LA() { return (uint64_t*)(smem + L.off); }  // [kDL+1] line start (abs)
    __device__ __forceinline__ uint64_t* LB() { return (uint64_t*)(smem + L.off) + (kDL + 1); }
    __device__ __forceinline__ uint32_t* MISC() { return (uint32_t*)(smem + L.misc); }
    __device__ __forceinline__ uint8_t* STAGE() { return smem + L.stage; }

    // One pass over the bytes [cb_lo, cb_hi) of lines [b0, b1) (Sec. IV-D-2: a
    // byte is a literal iff an odd run of spaces precedes it; a code expands to
    // its dictionary string).  Every line ends with its newline in CB.  Gives
    // each byte its output length and records line ends (batch-relative) in
    // LLEN.  With emit, the output bytes go to STAGE at index sbase + position;
    // bytes whose index falls outside [0, kDStage) are left out and set *spill.
    // Lines marked in BAD produce only their newline when mask_bad is set.
    // Bytes that make a line corrupt mark it in BAD and set *err.  Returns the
    // output bytes of the batch.
    //
    // clean: the batch has no bad line and exactly one newline per line, so the
    // lines end at the newlines: line indices come from a count of newlines, and
    // a piece with no space and no escape reaching into it is measured with
    // byte-parallel arithmetic.
    __device__ __forceinline__ uint32_t pass(uint32_t b0, uint32_t b1, uint32_t cb_lo, uint32_t cb_hi, bool mask_bad,
                                             bool emit, int32_t sbase, bool* err, bool* spill, bool clean) {
        const uint32_t tid = threadIdx.x;
        const uint8_t* cb = CB();
        const uint32_t* qoff = QOFF();
        uint8_t* bad = BAD();
        uint32_t* llen = LLEN();
        uint8_t* stage = STAGE();
        uint32_t* psc = MISC() + kDmScanA;
        uint32_t carry_pos = 0, carry_nl = 0;
        bool err_any = false, spill_any = false;
        const uint32_t c0 = cb_lo & ~15u;
        for (uint32_t seg = c0; seg < cb_hi; seg += kSeg) {
            const uint32_t x0 = seg + tid * 16;
            uint4 w4 = make_uint4(0, 0, 0, 0);
            if (x0 < cb_hi) w4 = *(const uint4*)(cb + x0);
            const uint32_t wv[4] = {w4.x, w4.y, w4.z, w4.w};
#define ZS_BYTE(k) ((wv[(k) >> 2] >> (8 * ((k) & 3))) & 0xFFu)
            // bytes of the chunk inside [cb_lo, cb_hi).  The clamps are signed: the
            // form  a < b ? b - a : 0  in unsigned arithmetic was turned into an
            // unconditional no-wrap subtraction, from which the optimizer
            // concluded a <= b on every lane.
            uint32_t valid = 0;
            {
                const uint32_t lo = (uint32_t)min(max((int32_t)cb_lo - (int32_t)x0, 0), 16);
                const uint32_t hi = (uint32_t)min(max((int32_t)cb_hi - (int32_t)x0, 0), 16);
                if (hi > lo) valid = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
            }
            uint32_t sp = 0;
            uint32_t lp[4] = {0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < 16; k++) {
                lp[k >> 2] |= (uint32_t)LEN[ZS_BYTE(k)] << (8 * (k & 3));
                sp |= (ZS_BYTE(k) == ' ' ? 1u : 0u) << k;
            }
            sp &= valid;
            // the run of spaces just before x0, read back from CB (lines end
            // with a newline, so a run never reaches into the previous line)
            uint32_t r = 0;
            if (valid && x0 > cb_lo) {
                for (uint32_t y = x0 - 16;; y -= 16) {
                    const uint4 p4 = *(const uint4*)(cb + y);
                    const uint32_t pw[4] = {p4.x, p4.y, p4.z, p4.w};
                    uint32_t ps = 0;
#pragma unroll
                    for (int k = 0; k < 16; k++)
                        ps |= ((((pw[k >> 2] >> (8 * (k & 3))) & 0xFFu) == ' ' && y + k >= cb_lo) ? 1u : 0u) << k;
                    const uint32_t tr = (uint32_t)__builtin_clz(~(ps << 16));
                    r += tr;
                    if (tr < 16 || y <= cb_lo) break;
                }
            }
            uint32_t sum = 0, term = 0, lit = 0, qfirst = b0, errm_pending = 0;
            bool swar = false;  // lengths from the byte-parallel path: no escape in the piece
            if (clean) {
                uint32_t errm = 0;
                if (sp == 0 && !(r & 1)) {
                    swar = true;
                    // no escape: byte-parallel lengths, newlines, undefined codes
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const uint32_t vb = (valid >> (4 * i)) & 0xFu;
                        const uint32_t vm = ((vb * 0x00204081u) & 0x01010101u) * 0xFFu;
                        const uint32_t nlw = swar_eq_bytes(wv[i], 0x0A0A0A0Au) & vm & 0x80808080u;
                        const uint32_t nl1 = nlw >> 7;
                        const uint32_t lenw = ((lp[i] & ~(nl1 * 0xFFu)) | nl1) & vm;
                        const uint32_t erw = swar_eq_bytes(lp[i], 0u) & ~nlw & vm & 0x80808080u;
                        lp[i] = lenw;
                        sum += (lenw * 0x01010101u) >> 24;
                        term |= ((nl1 | (nl1 >> 7) | (nl1 >> 14) | (nl1 >> 21)) & 0xFu) << (4 * i);
                        const uint32_t e1 = erw >> 7;
                        errm |= ((e1 | (e1 >> 7) | (e1 >> 14) | (e1 >> 21)) & 0xFu) << (4 * i);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        const bool isv = (valid >> k) & 1;
                        const uint32_t ck = ZS_BYTE(k);
                        const uint32_t tl = (lp[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                        const bool iss = (sp >> k) & 1;
                        const bool ist = isv && ck == '\n';
                        const bool islit = isv && (r & 1);
                        uint32_t len;
                        bool e = false;
                        if (!isv) len = 0;
                        else if (ist) { len = 1; e = islit; }
                        else if (islit) { len = 1; e = ck < 0x20u || ck > 0x7Eu; }
                        else if (iss) len = 0;
                        else { len = tl; e = tl == 0; }
                        errm |= (e ? 1u : 0u) << k;
                        term |= (ist ? 1u : 0u) << k;
                        lit |= (islit && !ist ? 1u : 0u) << k;
                        lp[k >> 2] = (lp[k >> 2] & ~(0xFFu << (8 * (k & 3)))) | (len << (8 * (k & 3)));
                        sum += len;
                        r = iss ? r + 1 : 0u;
                    }
                }
                if (errm) {
                    err_any = true;  // lines marked once the newlines before each byte are known
                    errm_pending = errm;
                }
            } else {
                // the line of the first valid byte
                uint32_t q = b0, nb = 0;
                if (valid) {
                    const uint32_t xs = x0 + (uint32_t)__builtin_ctz(valid);  // the first valid byte
                    uint32_t l = b0, h = b1;
                    while (h - l > 1) {
                        const uint32_t mid = (l + h) >> 1;
                        if (qoff[mid] <= xs) l = mid;
                        else h = mid;
                    }
                    q = l;
                    nb = qoff[q + 1];
                }
                qfirst = q;
                bool qbad = mask_bad && valid && bad[q] != 0;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    const uint32_t x = x0 + k;
                    const bool isv = (valid >> k) & 1;
                    if (isv && x >= nb) {
                        do {
                            q++;
                            nb = qoff[q + 1];
                        } while (x >= nb);
                        qbad = mask_bad && bad[q] != 0;
                    }
                    const uint32_t ck = ZS_BYTE(k);
                    const uint32_t tl = (lp[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                    const bool iss = (sp >> k) & 1;
                    const bool ist = isv && (x + 1 == nb);
                    const bool islit = isv && (r & 1);
                    uint32_t len;
                    bool e = false;
                    if (!isv) len = 0;
                    else if (qbad) len = ist ? 1u : 0u;
                    else if (ist) { len = 1; e = islit; }                         // a dangling escape
                    else if (islit) { len = 1; e = ck < 0x20u || ck > 0x7Eu; }    // literal outside 0x20..0x7E
                    else if (iss) len = 0;
                    else { len = tl; e = tl == 0; }                              // undefined code
                    if (e) {
                        bad[q] = (uint8_t)kErrCorrupt;
                        err_any = true;
                    }
                    term |= (ist ? 1u : 0u) << k;
                    lit |= (islit && !ist ? 1u : 0u) << k;
                    lp[k >> 2] = (lp[k >> 2] & ~(0xFFu << (8 * (k & 3)))) | (len << (8 * (k & 3)));
                    sum += len;
                    r = iss ? r + 1 : 0u;
                }
            }
            uint32_t segtot;
            // clean batches: the newlines ride along in the scan (bits 18 and up)
            const uint32_t scan = block_excl_scan(clean ? (sum | ((uint32_t)__popc(term) << 18)) : sum, psc, &segtot);
            const uint32_t pos0 = carry_pos + (clean ? (scan & 0x3FFFFu) : scan);
            if (clean) {
                qfirst = b0 + carry_nl + (scan >> 18);
                if (errm_pending) {
                    for (uint32_t m = errm_pending; m; m &= m - 1) {
                        const uint32_t k = (uint32_t)__builtin_ctz(m);
                        bad[qfirst + __popc(term & ((1u << k) - 1u))] = (uint8_t)kErrCorrupt;
                    }
                }
                carry_nl += segtot >> 18;
                segtot &= 0x3FFFFu;
            }
            if (term) {
                uint32_t qq = qfirst, pos = pos0;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    pos += (lp[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                    if ((term >> k) & 1) llen[qq++] = pos;
                }
            }
            if (emit && sum) {
                const int32_t st0 = sbase + (int32_t)pos0;
                if (st0 >= 0 && st0 + (int32_t)sum <= kDStage && swar && lmax8) {
                    // every byte is a code of at most 8 bytes (a newline's row
                    // of EXP holds a newline; rows are zero past their length):
                    // the run is built with funnel shifts and stored by dwords,
                    // bytes only in the two dwords shared with the neighbours
                    uint32_t* st32 = (uint32_t*)stage;
                    const uint32_t s0 = (uint32_t)st0, lead = s0 & 3u, a0 = s0 >> 2;
                    uint32_t a = a0, p = lead, acc = 0;
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        const uint32_t len = (lp[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                        uint2 e = *(const uint2*)(EXP + ZS_BYTE(k) * kExpStride);
                        if (len == 0) e = make_uint2(0, 0);  // a byte outside the batch adds nothing
                        const uint32_t sh = 8 * p;
                        const uint32_t c0 = acc | (e.x << sh);
                        const uint32_t c1 = p ? __builtin_amdgcn_alignbit(e.y, e.x, 32 - sh) : e.y;
                        const uint32_t c2 = p ? (e.y >> (32 - sh)) : 0u;
                        const uint32_t n = p + len;
                        if (n >= 4) {
                            if (a == a0 && lead) {
                                for (uint32_t j = lead; j < 4; j++) stage[4 * a + j] = (uint8_t)(c0 >> (8 * j));
                            } else {
                                st32[a] = c0;
                            }
                        }
                        if (n >= 8) st32[a + 1] = c1;
                        acc = n >= 8 ? c2 : (n >= 4 ? c1 : c0);
                        a += n >> 2;
                        p = n & 3u;
                    }
                    for (uint32_t j = (a == a0 ? lead : 0u); j < p; j++) stage[4 * a + j] = (uint8_t)(acc >> (8 * j));
                } else if (st0 >= 0 && st0 + (int32_t)sum <= kDStage) {
                    StageWriter wr;
                    wr.begin(stage, (uint32_t)st0);
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        const uint32_t len = (lp[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                        if (len) {
                            const uint32_t ck = ZS_BYTE(k);
                            if (((term | lit) >> k) & 1) {
                                wr.add(((term >> k) & 1) ? (uint32_t)'\n' : ck, 1);
                            } else {
                                const uint2 e = *(const uint2*)(EXP + ck * kExpStride);
                                wr.add(e.x, min(len, 4u));
                                if (len > 4) wr.add(e.y, min(len - 4, 4u));
                                if (len > 8) {
                                    const uint2 f = *(const uint2*)(EXP + ck * kExpStride + 8);
                                    wr.add(f.x, min(len - 8, 4u));
                                    if (len > 12) wr.add(f.y, len - 12);
                                }
                            }
                        }
                    }
                    wr.finish();
                } else {
                    // part of this thread's bytes lies outside the stage window
                    spill_any = true;
                    int32_t sx = st0;
#pragma unroll 1
                    for (int k = 0; k < 16; k++) {
                        const uint32_t len = (lp[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                        const uint32_t ck = (wv[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                        for (uint32_t j = 0; j < len; j++, sx++) {
                            if (sx < 0 || sx >= kDStage) continue;
                            uint32_t b;
                            if ((term >> k) & 1) b = '\n';
                            else if ((lit >> k) & 1) b = ck;
                            else b = EXP[ck * kExpStride + j];
                            stage[sx] = (uint8_t)b;
                        }
                    }
                }
            }
#undef ZS_BYTE
            carry_pos += segtot;
        }
        *err = __syncthreads_or(err_any) != 0;
        if (spill) *spill = __syncthreads_or(spill_any) != 0;
        return carry_pos;
    }

    // Size a loaded batch: one pass, and a second one with the lines found
    // corrupt masked.  Reports the corrupt lines.
    __device__ __forceinline__ uint32_t size_batch(uint32_t b0, uint32_t b1, uint32_t cb_lo, uint32_t cb_hi,
                                                   bool anybad, bool clean) {
        bool err;
        uint32_t T = pass(b0, b1, cb_lo, cb_hi, anybad, false, 0, &err, nullptr, clean);
        if (err) {
            T = pass(b0, b1, cb_lo, cb_hi, true, false, 0, &err, nullptr, false);
            const uint32_t q = b0 + threadIdx.x;
            if (q < b1 && BAD()[q] == kErrCorrupt) note_error(A.ws, r0 + q, kErrCorrupt);
        }
        __syncthreads();
        return T;
    }

    // Decode a loaded batch into out[g0, ...): passes that write the stage,
    // flushed with 16-byte stores on the destination's 16-byte grid; a batch
    // whose output exceeds the stage goes out in several windows.  Returns the
    // batch's output bytes; line ends are left in LLEN.
    __device__ __forceinline__ uint32_t decode_batch(uint32_t b0, uint32_t b1, uint32_t cb_lo, uint32_t cb_hi,
                                                     bool anybad, bool clean, uint64_t g0, bool write) {
        bool err, spill;
        const uintptr_t dst = (uintptr_t)(A.out + g0);
        const uintptr_t a0 = dst & ~(uintptr_t)15;
        const int32_t lead = (int32_t)(dst - a0);
        uint32_t T = pass(b0, b1, cb_lo, cb_hi, anybad, write, lead, &err, &spill, clean);
        if (err) {
            T = pass(b0, b1, cb_lo, cb_hi, true, write, lead, &err, &spill, false);
            const uint32_t q = b0 + threadIdx.x;
            if (q < b1 && BAD()[q] == kErrCorrupt) note_error(A.ws, r0 + q, kErrCorrupt);
        }
        if (!write) {
            __syncthreads();
            return T;
        }
        uint8_t* stage = STAGE();
        // window w holds destination bytes [a0 + w kDStage, a0 + (w + 1) kDStage)
        for (uint32_t w = 0;; w++) {
            const uint64_t wlo = (uint64_t)w * kDStage;  // relative to a0
            if (w > 0) pass(b0, b1, cb_lo, cb_hi, true, true, lead - (int32_t)wlo, &err, &spill, false);
            const int64_t wrel = (int64_t)wlo - lead;  // batch position of the window's first byte
            uint64_t lo = (uint64_t)max(wrel, (int64_t)0), hi = (uint64_t)(wrel + kDStage);
            if (hi > T) hi = T;
            __syncthreads();
            flush_stage(A.out, g0 + lo, g0 + hi, a0 + (uintptr_t)wlo, stage);
            __syncthreads();
            if (!spill || hi >= T) break;
        }
        return T;
    }

    // Framing of the requests of tile t; returns the number of lines and sets
    // *regular (no framing error in the tile).
    __device__ __forceinline__ uint32_t setup_tile(uint32_t t, bool* regular) {
        const uint32_t tid = threadIdx.x;
        const bool gather = A.ids != nullptr;
        uint8_t* bad = BAD();
        uint64_t* la = LA();
        uint64_t* lb = LB();
        r0 = (uint64_t)t * A.tl;
        const uint32_t nl = (uint32_t)min((uint64_t)A.tl, A.nreq - r0);
        if (tid < nl) {
            const uint64_t r = r0 + tid;
            uint32_t fe = 0;
            const uint64_t id = gather ? A.ids[r] : r;
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
        }
        *regular = __syncthreads_and(tid >= nl || bad[tid] == 0) != 0;
        return nl;
    }

    // Output offsets of lines [b0, b1) whose batch starts at global offset g.
    __device__ __forceinline__ void write_offsets(uint32_t b0, uint32_t b1, uint64_t g) {
        const uint32_t q = b0 + threadIdx.x;
        if (q < b1) A.out_off[r0 + q + 1] = g + LLEN()[q];
    }

    // Tiles in ticket order, each placed by a decoupled look-back once its
    // size is known.  A tile decoded in one pass publishes its size and keeps
    // its bytes in the stage; it is placed one step later, after the next
    // tile's framing and load, so that its predecessors have had time to
    // publish and the workgroup does not wait on them.
    __device__ __forceinline__ void run_lookback() {
        uint32_t* misc = MISC();
        uint32_t* llen = LLEN();
        const uint32_t tid = threadIdx.x;
        const bool gather = A.ids != nullptr;
        bool pend = false;
        uint32_t pt = 0, pT = 0, pnl = 0;
        uint64_t pr0 = 0;
        // with at most one tile per workgroup nothing is gained by waiting
        const bool defer = A.ntiles > gridDim.x;
        // the first ticket was claimed in the kernel's prologue
        uint32_t next = misc[kDmSlot];
        bool claimed = true;
        // place the pending tile: its line ends are still in LLEN, its bytes in the stage
        auto place_pending = [&]() {
            if (tid < 64) {
                const uint64_t ex = lookback_walk(A.status, pt, pT);
                if (tid == 0) ((uint64_t*)misc)[kDmBase64 / 2] = ex;
            }
            __syncthreads();
            const uint64_t gbase = ((uint64_t*)misc)[kDmBase64 / 2];
            if (pt == 0 && tid == 0) A.out_off[0] = 0;
            if (tid < pnl) A.out_off[pr0 + tid + 1] = gbase + llen[tid];
            const bool fits = gbase + pT <= A.out_cap;
            if (!fits && tid == 0) atomicOr(&A.ws->enospc, 1u);
            if (fits) copy_slot_direct(A.out, STAGE(), pT, gbase);
            __syncthreads();
            pend = false;
        };
        while (true) {
            // with one workgroup per tile (the grid is never larger than the
            // tile count) every workgroup's first ticket was its only tile
            const uint32_t t = claimed ? next : gridDim.x >= A.ntiles ? A.ntiles : claim_tile(A.ws, &misc[kDmSlot]);
            claimed = false;
            if (t >= A.ntiles) {
                if (pend) place_pending();
                break;
            }
            bool regular;
            const uint32_t nl = setup_tile(t, &regular);
            if (A.out) {
                // the usual tile, one batch: lengths and bytes in one pass, the
                // bytes at tile-relative stage positions, copied out shifted to
                // the tile's alignment once it is placed
                uint32_t b1, lo, hi;
                bool anybad, clean, err, spill;
                load_batch(0, nl, regular, gather, &b1, &lo, &hi, &anybad, &clean);
                if (pend) place_pending();
                if (b1 == nl) {
                    uint32_t T = pass(0, nl, lo, hi, anybad, true, 0, &err, &spill, clean);
                    if (err) {
                        T = pass(0, nl, lo, hi, true, true, 0, &err, &spill, false);
                        if (tid < nl && BAD()[tid] == kErrCorrupt) note_error(A.ws, r0 + tid, kErrCorrupt);
                        anybad = true;
                        clean = false;
                    }
                    if (!spill && defer) {
                        if (tid == 0) publish_aggregate(A.status, t, T);
                        pend = true;
                        pt = t;
                        pT = T;
                        pnl = nl;
                        pr0 = r0;
                        continue;
                    }
                    // placed at once; more output than the stage holds goes out in windows
                    if (tid < 64) {
                        const uint64_t ex = lookback(A.status, t, T);
                        if (tid == 0) ((uint64_t*)misc)[kDmBase64 / 2] = ex;
                    }
                    __syncthreads();
                    const uint64_t gbase = ((uint64_t*)misc)[kDmBase64 / 2];
                    if (t == 0 && tid == 0) A.out_off[0] = 0;
                    write_offsets(0, nl, gbase);
                    const bool fits = gbase + T <= A.out_cap;
                    if (!fits && tid == 0) atomicOr(&A.ws->enospc, 1u);
                    if (fits) {
                        if (!spill) {
                            copy_slot_direct(A.out, STAGE(), T, gbase);
                        } else {
                            __syncthreads();
                            decode_batch(0, nl, lo, hi, anybad, clean, gbase, true);
                        }
                    }
                    __syncthreads();
                    continue;
                }
                __syncthreads();
            }
            uint32_t tpos = 0, b0 = 0, nb = 0, T = 0, lo = 0, hi = 0, lb1 = 0;
            bool lbad = false, lclean = false;
            while (b0 < nl) {
                uint32_t b1;
                bool anybad, clean;
                load_batch(b0, nl, regular, gather, &b1, &lo, &hi, &anybad, &clean);
                T = size_batch(b0, b1, lo, hi, anybad, clean);
                lb1 = b1;
                lbad = anybad;
                lclean = clean;
                // line ends relative to the tile
                const uint32_t q = b0 + tid;
                if (q < b1) llen[q] += tpos;
                __syncthreads();
                tpos += T;
                b0 = b1;
                nb++;
            }
            if (tid < 64) {
                const uint64_t ex = lookback(A.status, t, tpos);
                if (tid == 0) ((uint64_t*)misc)[kDmBase64 / 2] = ex;
            }
            __syncthreads();
            const uint64_t gbase = ((uint64_t*)misc)[kDmBase64 / 2];
            if (t == 0 && tid == 0) A.out_off[0] = 0;
            write_offsets(0, nl, gbase);
            const bool fits = gbase + tpos <= A.out_cap;
            if (!fits && tid == 0) atomicOr(&A.ws->enospc, 1u);
            if (A.out && fits) {
                if (nb == 1) {
                    __syncthreads();
                    decode_batch(0, lb1, lo, hi, lbad, lclean, gbase, true);
                } else {
                    uint32_t g = 0;
                    b0 = 0;
                    while (b0 < nl) {
                        uint32_t b1;
                        bool anybad, clean;
                        load_batch(b0, nl, regular, gather, &b1, &lo, &hi, &anybad, &clean);
                        g += decode_batch(b0, b1, lo, hi, anybad, clean, gbase + g, true);
                        b0 = b1;
                        __syncthreads();
                    }
                }
            }
            __syncthreads();
        }
    }

    // Gather of a batch whose lines are all short: lane q copies line q into CB
    // at pos from the aligned dwords that hold it, all of them loaded before
    // the first is used.  Returns false, having written nothing, when a line of
    // the batch is longer than kLaneLine bytes or its dwords would reach outside
    // [in, in + in_bytes); the caller then gathers by 16-byte chunks.
    static constexpr uint32_t kLaneLine = 64;
    static constexpr int kLaneDw = 17;  // dwords that hold kLaneLine bytes at any alignment
    __device__ __forceinline__ bool gather_lanes(uint32_t q, uint32_t b0, uint32_t b1, uint32_t sz, uint32_t pos) {
        const uint8_t* bad = BAD();
        const uint64_t* la = LA();
        const uint64_t* lb = LB();
        uint8_t* cb = CB();
        const bool mine = q >= b0 && q < b1;
        const bool isbad = mine && bad[q] != 0;
        // bytes of the line in memory (a virtual last newline is not)
        uint32_t nreal = 0;
        uintptr_t d0 = 0;
        int ndw = 0;
        bool ok = true;
        if (mine && !isbad) {
            nreal = (lb[q] == A.in_bytes + 1) ? sz - 1 : sz;
            if (nreal > 0) {
                const uintptr_t first = (uintptr_t)(A.in + la[q]);
                d0 = first & ~(uintptr_t)3;
                const uintptr_t dl = (first + nreal - 1) & ~(uintptr_t)3;
                ndw = (int)((dl - d0) >> 2) + 1;
                ok = nreal <= kLaneLine && d0 >= (uintptr_t)A.in && dl + 4 <= (uintptr_t)(A.in + A.in_bytes);
            }
        }
        if (__syncthreads_or(!ok) != 0) return false;
        if (nreal > 0) {
            // pointer arithmetic on A.in (not integers) keeps these global loads
            const uint8_t* first = A.in + la[q];
            const int sh = (int)(((uintptr_t)first) & 3);
            const uint32_t* dw = (const uint32_t*)(first - sh);
            uint32_t w[kLaneDw];
#pragma unroll
            for (int k = 0; k < kLaneDw; k++) w[k] = dw[min(k, ndw - 1)];
            __builtin_amdgcn_sched_barrier(0);  // every load issued before the first store
#pragma unroll
            for (int k = 0; k < kLaneDw; k++) {
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const int idx = 4 * k + b - sh;
                    if (idx >= 0 && idx < (int)nreal) cb[pos + idx] = (uint8_t)(w[k] >> (8 * b));
                }
            }
        }
        // a bad line is a lone newline; a virtual newline is written here
        if (mine && (isbad || nreal < sz)) cb[pos + sz - 1] = '\n';
        __syncthreads();
        return true;
    }

    // Choose the batch [b0, b1) that fits the CB buffer and load it.  Lines are
    // packed at qoff[q]; every line ends with its newline in CB (a line whose
    // last byte is not a newline is bad, and its last CB byte is made one so
    // that escape runs never cross lines).
    __device__ __forceinline__ void load_batch(uint32_t b0, uint32_t nl, bool regular, bool gather, uint32_t* b1_out,
                                               uint32_t* cb_lo, uint32_t* cb_hi, bool* anybad, bool* clean) {
        const uint32_t tid = threadIdx.x;
        uint32_t* misc = MISC();
        uint8_t* bad = BAD();
        uint32_t* qoff = QOFF();
        uint64_t* la = LA();
        uint64_t* lb = LB();
        uint8_t* cb = CB();
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
            __syncthreads();
        } else if (gather_lanes(q, b0, b1, sz, pos)) {
            // every line of the batch was copied by its own lane
        } else {
            // gather: each thread fills 16-byte chunks of CB; the line of a
            // chunk's first byte comes from a search of qoff.  The source
            // addresses are found first (LDS only), then the 16 loads are
            // issued with no branch between them, so that they are all in
            // flight together (a load inside the per-byte branches was waited
            // for before the next one was issued)
            const uint32_t lo = qoff[b0], hi = qoff[b1];
            const bool has_in = A.in_bytes > 0;
            for (uint32_t x0 = (lo & ~15u) + tid * 16; x0 < hi; x0 += kWG * 16) {
                uint32_t l = b0, r = b1;
                const uint32_t xs = max(x0, lo);
                while (r - l > 1) {
                    const uint32_t mid = (l + r) >> 1;
                    if (qoff[mid] <= xs) l = mid;
                    else r = mid;
                }
                uint32_t qq = l;
                uint32_t nb = qoff[qq + 1];
                // per byte: kind (2 bits: 0 a byte of line qq at offset o, 1 a
                // newline, 2 zero) | qq << 2 (qq <= kDL) | o << 11 (o <= kMaxCLine)
                uint32_t pk[16];
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    const uint32_t x = x0 + k;
                    uint32_t e = 2;
                    if (x >= lo && x < hi) {
                        while (x >= nb) {
                            qq++;
                            nb = qoff[qq + 1];
                        }
                        if (bad[qq] || (x + 1 == nb && lb[qq] == A.in_bytes + 1)) {
                            // a bad line is a lone newline; a virtual newline is not in memory
                            e = (x + 1 == nb) ? 1u : 2u;
                        } else {
                            e = (qq << 2) | ((x - qoff[qq]) << 11);
                        }
                    }
                    pk[k] = e;
                }
                uint32_t v[16];
                if (has_in) {
                    // a byte that is not loaded reads A.in[0] (in bounds) instead
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        const uint32_t e = pk[k];
                        const uint64_t sa = (e & 3u) == 0 ? la[(e >> 2) & 511u] + (e >> 11) : 0;
                        v[k] = A.in[sa];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 16; k++) v[k] = 0;
                }
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    const uint32_t kd = pk[k] & 3u;
                    const uint8_t byte = kd == 0 ? (uint8_t)v[k] : kd == 1 ? (uint8_t)'\n' : (uint8_t)0;
                    if (x0 + k >= lo && x0 + k < hi) cb[x0 + k] = byte;
                }
            }
            __syncthreads();
        }
        // the newline must be where the index says
        bool isbad = false;
        if (q < b1) {
            if (!bad[q] && cb[qoff[q + 1] - 1] != '\n') {
                bad[q] = kErrInval;
                note_error(A.ws, r0 + q, kErrInval);
                cb[qoff[q + 1] - 1] = '\n';
            }
            isbad = bad[q] != 0;
        }
        *anybad = __syncthreads_or(isbad) != 0;
        // clean: no bad line and no newline inside a line (one newline per line)
        {
            const uint32_t lo = qoff[b0], hi = qoff[b1];
            uint32_t nnl = 0;
            for (uint32_t x0 = (lo & ~15u) + tid * 16; x0 < hi; x0 += kWG * 16) {
                const uint4 v = *(const uint4*)(cb + x0);
                const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 16; k++)
                    nnl += (x0 + k >= lo && x0 + k < hi && ((wv[k >> 2] >> (8 * (k & 3))) & 0xFFu) == '\n') ? 1u : 0u;
            }
            uint32_t tot;
            block_excl_scan(nnl, misc + kDmScanB, &tot);
            *clean = !*anybad && tot == b1 - b0;
        }
        *b1_out = b1;
        *cb_lo = qoff[b0];
        *cb_hi = qoff[b1];
    }
};

__global__ void __launch_bounds__(kWG) decompress_kernel(DecompressArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    {
        // the first tile's ticket is claimed while the tables load (the two
        // round trips overlap); it waits in the decoder's slot word
        uint32_t first = 0;
        if (threadIdx.x == 0) first = atomicAdd(&a.ws->ticket, 1u);
        // header + LEN at [0, 320), EXP at [320, 320 + 4096), in 16-byte pieces
        uint4* dst = (uint4*)smem;
        for (uint32_t k = threadIdx.x; k < (64 + 256 + 256 * kExpStride) / 16; k += kWG) {
            uint32_t src;
            if (k < 4) src = 16 * k;
            else if (k < 20) src = a.off_len + 16 * (k - 4);
            else src = a.off_exp + 16 * (k - 20);
            // the row of byte '\n' (never a code) holds a newline, for the
            // decoder's byte-parallel path
            dst[k] = (k == 20 + '\n') ? make_uint4('\n', 0, 0, 0) : *(const uint4*)(a.tables + src);
        }
        if (threadIdx.x == 0) ((uint32_t*)(smem + decompress_lds().misc))[kDmSlot] = first;
    }
    __syncthreads();
    Decoder d(a, smem);
    d.run_lookback();
}

// Exclusive prefix of n per-tile totals: base[i] = total[0] + ... + total[i-1],
// base[n] = the sum.  One workgroup of 1024 threads, each scanning a run of
// consecutive tiles.
constexpr int kScanWG = 1024;
__global__ void __launch_bounds__(kScanWG) tile_scan_kernel(const uint32_t* total, uint64_t* base, uint32_t n) {
    // blocks of kScanWG * kScanPer totals: each thread loads its kScanPer
    // neighbouring totals at once (all loads in flight together), the block is
    // scanned through the waves' sums, and the running carry moves to the next block
    constexpr uint32_t kScanPer = 16;
    __shared__ uint64_t wsum[kScanWG / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // 16-byte loads and stores where both arrays are 16-byte aligned (each thread's
    // first element is: kScanPer is a multiple of 4)
    const bool vec = (((uintptr_t)total | (uintptr_t)base) & 15u) == 0;
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < n; b0 += kScanWG * kScanPer) {
        const uint32_t i0 = b0 + tid * kScanPer;
        uint32_t v[kScanPer];
        uint64_t s = 0;
        if (vec && i0 + kScanPer <= n) {
#pragma unroll
            for (uint32_t j = 0; j < kScanPer; j += 4) {
                const uint4 q = *(const uint4*)(total + i0 + j);
                v[j] = q.x;
                v[j + 1] = q.y;
                v[j + 2] = q.z;
                v[j + 3] = q.w;
            }
        } else {
#pragma unroll
            for (uint32_t j = 0; j < kScanPer; j++) v[j] = i0 + j < n ? total[i0 + j] : 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < kScanPer; j++) s += v[j];
        const uint64_t inc = wave_incl_scan64(s);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint64_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < kScanWG / 64; k++) {
            const uint64_t x = wsum[k];
            before += ((uint32_t)k < w) ? x : 0ull;
            all += x;
        }
        uint64_t run = carry + before + inc - s;
        if (vec && i0 + kScanPer <= n) {
#pragma unroll
            for (uint32_t j = 0; j < kScanPer; j += 2) {
                const uint64_t r0 = run, r1 = run + v[j];
                run = r1 + v[j + 1];
                *(ulonglong2*)(base + i0 + j) = make_ulonglong2(r0, r1);
            }
        } else {
#pragma unroll
            for (uint32_t j = 0; j < kScanPer; j++) {
                if (i0 + j < n) base[i0 + j] = run;
                run += v[j];
            }
        }
        carry += all;
        __syncthreads();  // wsum is rewritten by the next block
    }
    if (tid == 0) base[n] = carry;
}

// ============================================================================
// Length-binned compression: device-side binning and placement
// ============================================================================

constexpr int kBinChunk = 4096;  // lines per workgroup of the binning kernels
constexpr uint32_t kMinLpt = 32;  // fewest lines per tile a bin may ask for (bounds the tile count)

struct BinArgs {
    const uint64_t* in_off;
    uint64_t n;
    uint64_t in_bytes;
    BinPlan* plan;
    uint32_t* hist;  // [chunk][kMaxBins]: counts, then (after the plan kernel) first positions
    uint32_t nchunks;
    uint32_t* ids;     // line ids in bin order
    uint32_t* pos_of;  // position of each line in that order
};

constexpr uint32_t kBinRows = kBinChunk / kWG;  // rows of kWG lines per chunk
static_assert(kBinRows * kWaves == 64, "one wave scans a bin's (row, wave) counts");

// The plan's bin bounds, read once per workgroup (uniform values).
struct BinBounds {
    uint32_t nb;
    uint32_t upper[kMaxBins];
    __device__ inline explicit BinBounds(const BinPlan* plan) {
        nb = plan->nbins;
#pragma unroll
        for (int i = 0; i < kMaxBins; i++) upper[i] = plan->upper[i];
    }
    // processing-order bin of the line [a, b) (bad framing: the last bin)
    __device__ inline uint32_t of(uint64_t a, uint64_t b, uint64_t in_bytes) const {
        if (b <= a || b > in_bytes + 1) return nb - 1;
        const uint64_t len = b - a - 1;
        uint32_t k = 0;
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)kMaxBins; i++) k += (i < nb && (uint64_t)upper[i] > len) ? 1u : 0u;
        return k == 0 ? 0u : k - 1;
    }
};

// The bins of this thread's line in every row of chunk c (kMaxBins past the end):
// every row's two offsets are loaded before the first bin is worked out.
__device__ inline void chunk_bins(const BinArgs& a, const BinBounds& bb, uint32_t c, uint32_t (&bins)[kBinRows]) {
    const uint64_t k0 = (uint64_t)c * kBinChunk;
    const uint64_t k1 = min(a.n, k0 + kBinChunk);
    uint64_t lo[kBinRows], hi[kBinRows];
#pragma unroll
    for (uint32_t r = 0; r < kBinRows; r++) {
        const uint64_t k = k0 + r * kWG + threadIdx.x;
        lo[r] = hi[r] = 0;
        if (k < k1) {
            lo[r] = a.in_off[k];
            hi[r] = a.in_off[k + 1];
        }
    }
#pragma unroll
    for (uint32_t r = 0; r < kBinRows; r++) {
        const uint64_t k = k0 + r * kWG + threadIdx.x;
        bins[r] = k < k1 ? bb.of(lo[r], hi[r], a.in_bytes) : (uint32_t)kMaxBins;
    }
}

// Counts of each bin per chunk of kBinChunk lines (one ballot per row and bin).
__global__ void __launch_bounds__(kWG) bin_count_kernel(BinArgs a) {
    __shared__ uint32_t cnt[kWaves][kMaxBins];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const BinBounds bb(a.plan);
    const uint32_t nb = bb.nb;
    for (uint32_t c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
        uint32_t bins[kBinRows];
        chunk_bins(a, bb, c, bins);
        for (uint32_t b = 0; b < nb; b++) {
            uint32_t m = 0;
#pragma unroll
            for (uint32_t r = 0; r < kBinRows; r++) m += (uint32_t)__popcll(__ballot(bins[r] == b));
            if (lane == 0) cnt[w][b] = m;
        }
        __syncthreads();
        if (tid < kMaxBins) {
            uint32_t v = 0;
            if (tid < nb)
                for (int ww = 0; ww < kWaves; ww++) v += cnt[ww][tid];
            a.hist[(size_t)c * kMaxBins + tid] = v;
        }
        __syncthreads();
    }
}

// One workgroup: bin sizes and starts, each chunk's first position per bin,
// the tiles of every bin.  Each thread takes a run of chunks: one pass sums its
// counts (both 16-byte halves of every row loaded at once), one block scan per
// bin, and a second pass writes the absolute first positions.
__global__ void __launch_bounds__(kWG) bin_plan_kernel(BinArgs a) {
    static_assert(kMaxBins == 8, "a histogram row is two 16-byte words");
    __shared__ uint32_t sc[kWaves + 1];
    __shared__ uint64_t bin_total[kMaxBins];
    __shared__ uint64_t bin_start[kMaxBins];
    BinPlan* plan = a.plan;
    const uint32_t tid = threadIdx.x;
    const uint32_t nb = plan->nbins;
    const uint32_t per = (a.nchunks + kWG - 1) / kWG;
    const uint32_t c0 = min(a.nchunks, tid * per), c1 = min(a.nchunks, c0 + per);
    uint4* rows = (uint4*)a.hist;  // row c: rows[2c], rows[2c + 1]
    uint32_t s[kMaxBins];
#pragma unroll
    for (int b = 0; b < kMaxBins; b++) s[b] = 0;
    for (uint32_t c = c0; c < c1; c++) {
        const uint4 x = rows[2 * c], y = rows[2 * c + 1];
        s[0] += x.x; s[1] += x.y; s[2] += x.z; s[3] += x.w;
        s[4] += y.x; s[5] += y.y; s[6] += y.z; s[7] += y.w;
    }
    uint32_t run[kMaxBins];
#pragma unroll
    for (uint32_t b = 0; b < (uint32_t)kMaxBins; b++) {
        run[b] = 0;
        if (b < nb) {  // uniform
            uint32_t tot;
            run[b] = block_excl_scan(s[b], sc, &tot);
            if (tid == 0) bin_total[b] = tot;
        }
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t start = 0;
        uint32_t tiles = 0;
        for (uint32_t b = 0; b < nb; b++) {
            plan->start[b] = start;
            plan->count[b] = (uint32_t)bin_total[b];
            plan->first_tile[b] = tiles;
            bin_start[b] = start;
            start += bin_total[b];
            tiles += (uint32_t)((bin_total[b] + plan->lpt[b] - 1) / plan->lpt[b]);
        }
        plan->first_tile[nb] = tiles;
    }
    __syncthreads();
    // chunk positions: absolute first position of every bin in every chunk
    uint32_t st[kMaxBins];
#pragma unroll
    for (uint32_t b = 0; b < (uint32_t)kMaxBins; b++) st[b] = b < nb ? (uint32_t)bin_start[b] + run[b] : 0u;
    for (uint32_t c = c0; c < c1; c++) {
        const uint4 x = rows[2 * c], y = rows[2 * c + 1];
        const uint32_t v[kMaxBins] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
        uint32_t o[kMaxBins];
#pragma unroll
        for (uint32_t b = 0; b < (uint32_t)kMaxBins; b++) {
            o[b] = b < nb ? st[b] : 0u;
            st[b] += v[b];
        }
        rows[2 * c] = make_uint4(o[0], o[1], o[2], o[3]);
        rows[2 * c + 1] = make_uint4(o[4], o[5], o[6], o[7]);
    }
}

// Stable scatter of the line ids into bin order: per chunk, every row's bin at
// once, a rank inside the wave from one ballot per row and bin, and one wave per
// bin scanning that bin's (row, wave) counts.
__global__ void __launch_bounds__(kWG) bin_scatter_kernel(BinArgs a) {
    __shared__ uint32_t cnt[kMaxBins][64];  // bin b, row r, wave w at [b][r * kWaves + w]
    __shared__ uint32_t run[kMaxBins];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const BinBounds bb(a.plan);
    const uint32_t nb = bb.nb;
    for (uint32_t c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
        const uint64_t k0 = (uint64_t)c * kBinChunk;
        const uint64_t k1 = min(a.n, k0 + kBinChunk);
        uint32_t bins[kBinRows], rank[kBinRows];
        chunk_bins(a, bb, c, bins);
#pragma unroll
        for (uint32_t r = 0; r < kBinRows; r++) rank[r] = 0;
        for (uint32_t b = 0; b < nb; b++) {
#pragma unroll
            for (uint32_t r = 0; r < kBinRows; r++) {
                const uint64_t m = __ballot(bins[r] == b);
                if (bins[r] == b) rank[r] = (uint32_t)__popcll(m & below);
                if (lane == 0) cnt[b][r * kWaves + w] = (uint32_t)__popcll(m);
            }
        }
        if (tid < kMaxBins) run[tid] = a.hist[(size_t)c * kMaxBins + tid];
        __syncthreads();
        // exclusive prefix of each bin's counts in (row, wave) order = line order
        for (uint32_t b = w; b < nb; b += kWaves) {
            const uint32_t v = cnt[b][lane];
            cnt[b][lane] = wave_incl_scan(v) - v;
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < kBinRows; r++) {
            const uint64_t k = k0 + r * kWG + tid;
            if (k < k1) {
                const uint32_t b = bins[r];
                const uint32_t pos = run[b] + cnt[b][r * kWaves + w] + rank[r];
                a.ids[pos] = (uint32_t)k;
                a.pos_of[k] = pos;
            }
        }
        __syncthreads();  // run and cnt are rewritten for the next chunk
    }
}

struct PlaceArgs {
    const uint32_t* pos_of;
    const uint64_t* soff;   // per line in bin order: staging start << 16 | compressed length
    const uint8_t* staging;
    uint64_t staging_bytes;
    uint64_t n;
    uint8_t* out;
    uint64_t out_cap;
    uint64_t* out_off;
    uint32_t ntiles;
    uint32_t* tile_total;
    const uint64_t* tile_base;
    WsHeader* ws;      // errors and ENOSPC (shared with the compression launches)
};

// Output bytes per tile of kCL lines in input order: a workgroup takes
// kCountTiles tiles per round, all their lines' descriptors loaded at once.
constexpr uint32_t kCountTiles = 4;
__global__ void __launch_bounds__(kWG) place_count_kernel(PlaceArgs a) {
    __shared__ uint32_t sc[kCountTiles][kWaves];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (uint32_t t0 = blockIdx.x * kCountTiles; t0 < a.ntiles; t0 += gridDim.x * kCountTiles) {
        uint32_t p[kCountTiles];
        bool in[kCountTiles];
#pragma unroll
        for (uint32_t j = 0; j < kCountTiles; j++) {
            const uint64_t k = (uint64_t)(t0 + j) * kCL + tid;
            in[j] = t0 + j < a.ntiles && k < a.n;
            p[j] = in[j] ? a.pos_of[k] : 0u;
        }
        uint64_t v[kCountTiles];
#pragma unroll
        for (uint32_t j = 0; j < kCountTiles; j++) v[j] = in[j] ? a.soff[p[j]] : 0ull;
#pragma unroll
        for (uint32_t j = 0; j < kCountTiles; j++) {
            const uint32_t s = (uint32_t)wave_sum64(v[j] & 0xFFFFu);
            if (lane == 0) sc[j][w] = s;
        }
        __syncthreads();
        if (tid < kCountTiles && t0 + tid < a.ntiles)
            a.tile_total[t0 + tid] = sc[tid][0] + sc[tid][1] + sc[tid][2] + sc[tid][3];
        __syncthreads();
    }
}

// Offsets in input order, and the lines' bytes from the staging area: each
// thread builds 16 bytes of the destination's 16-byte grid - the first line
// from a search of the tile's line starts, each line the piece overlaps from two
// aligned 16-byte loads of the staging copy shifted into place (byte by byte
// where those loads would leave the staging area) - and stores them at once.
__global__ void __launch_bounds__(kWG) place_write_kernel(PlaceArgs a) {
    __shared__ uint32_t e[kCL + 1];
    __shared__ uint64_t src[kCL];
    __shared__ uint32_t sc[kWaves + 1];
    const uint32_t tid = threadIdx.x;
    for (uint32_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const uint64_t k0 = (uint64_t)t * kCL;
        const uint32_t nl = (uint32_t)min((uint64_t)kCL, a.n - k0);
        uint32_t len = 0;
        if (tid < nl) {
            const uint32_t p = a.pos_of[k0 + tid];
            src[tid] = a.soff[p] >> 16;
            len = (uint32_t)(a.soff[p] & 0xFFFFu);
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan(len, sc, &tot);
        const uint64_t base = a.tile_base[t];
        if (tid < nl) {
            e[tid] = ex;
            a.out_off[k0 + tid + 1] = base + ex + len;
        }
        if (tid == 0) {
            e[nl] = tot;
            if (t == 0) a.out_off[0] = 0;
        }
        __syncthreads();
        const bool fits = base + tot <= a.out_cap;
        if (!fits && tid == 0) atomicOr(&a.ws->enospc, 1u);
        if (a.out && fits && tot) {
            const uintptr_t dst = (uintptr_t)(a.out + base);
            const uintptr_t a0 = dst & ~(uintptr_t)15;
            const uint32_t lead = (uint32_t)(dst - a0);
            const uint32_t nch = (lead + tot + 15) >> 4;
            const uintptr_t sb = (uintptr_t)a.staging, se = sb + a.staging_bytes;
            for (uint32_t c = tid; c < nch; c += kWG) {
                const int32_t p0 = (int32_t)(c * 16) - (int32_t)lead;  // tile position of the chunk's byte 0
                const uint32_t plo = (uint32_t)max(p0, 0), phi = (uint32_t)min(p0 + 16, (int32_t)tot);
                uint32_t l = 0, h = nl;
                while (h - l > 1) {
                    const uint32_t mid = (l + h) >> 1;
                    if (e[mid] <= plo) l = mid;
                    else h = mid;
                }
                uint32_t q = l;
                uint32_t wv[4] = {0, 0, 0, 0};
                while (true) {
                    // chunk bytes [k0, k1) are line q's bytes from tile position s0
                    const uint32_t qs = e[q], qe = e[q + 1];
                    const uint32_t s0 = max(qs, plo), s1 = min(qe, phi);
                    const uint32_t k0 = (uint32_t)((int32_t)s0 - p0), k1 = (uint32_t)((int32_t)s1 - p0);
                    const uintptr_t sa = sb + src[q] + (s0 - qs);
                    const uintptr_t c0 = sa & ~(uintptr_t)15;
                    if (c0 >= sb && c0 + 32 <= se) {
                        or_shifted_piece(wv, sa, k0, k1);
                    } else {
                        for (uint32_t k = k0; k < k1; k++) {
                            const uintptr_t b = sa + (k - k0);
                            if (b < se) wv[k >> 2] |= (uint32_t)(*(const uint8_t*)b) << (8 * (k & 3));
                        }
                    }
                    if (qe >= phi) break;
                    q++;
                }
                uint8_t* d = (uint8_t*)(a0 + ((uintptr_t)c << 4));
                if (p0 >= 0 && p0 + 16 <= (int32_t)tot) {
                    *(uint4*)d = make_uint4(wv[0], wv[1], wv[2], wv[3]);
                } else {
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        const int32_t p = p0 + k;
                        if (p >= 0 && p < (int32_t)tot) d[k] = (uint8_t)(wv[k >> 2] >> (8 * (k & 3)));
                    }
                }
            }
        }
        __syncthreads();
    }
}

// A call's result, after its last kernel: the workgroups do not count
// themselves out (one contended atomic each at the end of every launch).
__global__ void result_kernel(WsHeader* h, ResultOut* res) {
    if (threadIdx.x == 0) write_result(h, res);
}

static zs_status launch_result(WsHeader* h, zs_result* res, hipStream_t s) {
    if (res) hipLaunchKernelGGL(result_kernel, dim3(1), dim3(64), 0, s, h, (ResultOut*)res);
    return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
}

// Zero the headers and the plan's counters; the plan's bins from the host's
// configuration.
struct BinInit {
    uint32_t nbins;
    uint32_t upper[kMaxBins];
    uint32_t lpt[kMaxBins];
};
__global__ void binned_init_kernel(WsHeader* h1, WsHeader* h2, BinPlan* plan, BinInit cfg, ResultOut* res) {
    const uint32_t i = threadIdx.x;
    if (i == 0) {
        WsHeader* hs[2] = {h1, h2};
        for (int j = 0; j < 2; j++) {
            hs[j]->ticket = 0;
            hs[j]->done = 0;
            hs[j]->enospc = 0;
            hs[j]->errkey = ~0ull;
            hs[j]->total = 0;
            hs[j]->alloc = 0;
        }
        plan->nbins = cfg.nbins;
        if (res) {
            res->code = 0;
            res->reserved = 0;
            res->first_bad = -1;
        }
    }
    if (i < kMaxBins) {
        plan->upper[i] = cfg.upper[i];
        plan->lpt[i] = cfg.lpt[i];
        plan->ticket[i] = 0;
    }
}

// ============================================================================
// Line index
// ============================================================================

constexpr int kIdxRounds = 8;                    // 16-byte loads per thread per tile
constexpr int kIdxTile = kWG * 16 * kIdxRounds;  // bytes per tile (32 KiB)

struct IndexArgs {
    const uint8_t* buf;
    uint64_t len;
    uint64_t* off;
    uint64_t off_cap;
    uint64_t* n_lines_out;
    uint32_t ntiles;
    WsHeader* ws;
    uint64_t* status;  // look-back words, one per tile (newline counts)
};

// per 4-byte word: bit 7 of each byte set where the byte is a newline (exact,
// no carries between bytes)
__device__ inline uint32_t newline_bits(uint32_t w) {
    const uint32_t x = w ^ 0x0A0A0A0Au;
    const uint32_t nz = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
    return ~nz & 0x80808080u;
}

// 16 bytes at x, bytes past len read as spaces
__device__ inline uint4 load16_or_pad(const uint8_t* buf, uint64_t len, uint64_t x, bool aligned) {
    if (aligned && x + 16 <= len) return *(const uint4*)(buf + x);
    uint32_t w[4] = {0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u};
    for (int b = 0; b < 16; b++)
        if (x + b < len) {
            const uint32_t sh = 8 * (b & 3);
            w[b >> 2] = (w[b >> 2] & ~(0xFFu << sh)) | ((uint32_t)buf[x + b] << sh);
        }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// The newline flags (bit 7 of each byte, from newline_bits) of a 4-byte word
// as 4 bits: a multiply gathers bits 0, 8, 16, 24 at bits 21..24 (no two
// partial products overlap).
__device__ inline uint32_t compact4(uint32_t nl) { return (((nl >> 7) * 0x00204081u) >> 21) & 0xFu; }

constexpr int kIdxLdsCap = kIdxTile / 4;  // newline positions of a tile staged in LDS (u16 each)

// One pass over the buffer.  Tiles are taken in ticket order; round k of a tile
// covers bytes [4096 k, 4096 k + 4096), 16 per thread, so every load is
// coalesced, and each round's newlines are kept as a 16-bit mask.  A tile
// publishes its newline count for a decoupled look-back and ranks its newlines
// into LDS (two buffers); it is placed one step later, after the next tile has
// been read, and its offsets go out as one contiguous, coalesced run.  A tile
// with more newlines than the LDS holds is placed at once and written from its
// masks.
__global__ void __launch_bounds__(kWG) index_kernel(IndexArgs a) {
    __shared__ uint32_t sc[kWaves][kIdxRounds];
    __shared__ uint16_t pos[2][kIdxLdsCap];
    __shared__ uint32_t slot;
    __shared__ uint64_t sbase_sh;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const bool aligned = (((uintptr_t)a.buf) & 15) == 0;
    bool pend = false;
    uint32_t pt = 0, ptot = 0, pb = 0, cur = 0;
    // after the last tile is placed: the virtual final newline, off[0], the count
    auto finish_last = [&](uint64_t sbase, uint32_t tot) {
        if (tid == 0) {
            uint64_t lines = sbase + tot;
            if (a.buf[a.len - 1] != '\n') {
                lines++;
                if (lines < a.off_cap) a.off[lines] = a.len + 1;
            }
            if (a.off_cap > 0) a.off[0] = 0;
            *a.n_lines_out = lines;
            if (lines + 1 > a.off_cap) atomicOr(&a.ws->enospc, 1u);
        }
    };
    auto place_pending = [&]() {
        if (tid < 64) {
            const uint64_t ex = lookback_walk(a.status, pt, ptot);
            if (tid == 0) sbase_sh = ex;
        }
        __syncthreads();
        const uint64_t sbase = sbase_sh;
        const uint64_t tb = (uint64_t)pt * kIdxTile;
        for (uint32_t i = tid; i < ptot; i += kWG) {
            const uint64_t k1 = sbase + 1 + i;
            if (k1 < a.off_cap) a.off[k1] = tb + pos[pb][i];
        }
        if (pt + 1 == a.ntiles) finish_last(sbase, ptot);
        pend = false;
        __syncthreads();  // sbase_sh is read by every wave before it is written again
    };
    while (true) {
        const uint32_t t = claim_tile(a.ws, &slot);
        if (t >= a.ntiles) {
            if (pend) place_pending();
            break;
        }
        const uint64_t tb = (uint64_t)t * kIdxTile;
        uint32_t m16[kIdxRounds], ex[kIdxRounds];
        uint4 v[kIdxRounds];
        if (aligned && tb + kIdxTile <= a.len) {  // the whole tile in bounds: plain loads
#pragma unroll
            for (int k = 0; k < kIdxRounds; k++) v[k] = *(const uint4*)(a.buf + tb + 4096u * k + 16u * tid);
        } else {  // the last tile or an unaligned buffer: one round at a time
#pragma unroll
            for (int k = 0; k < kIdxRounds; k++) {
                v[k] = load16_or_pad(a.buf, a.len, tb + 4096u * k + 16u * tid, aligned);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int k = 0; k < kIdxRounds; k++)
            m16[k] = compact4(newline_bits(v[k].x)) | (compact4(newline_bits(v[k].y)) << 4) |
                     (compact4(newline_bits(v[k].z)) << 8) | (compact4(newline_bits(v[k].w)) << 12);
#pragma unroll
        for (int k = 0; k < kIdxRounds; k++) {
            const uint32_t c = __popc(m16[k]);
            const uint32_t inc = wave_incl_scan(c);
            ex[k] = inc - c;
            if (lane == 63) sc[w][k] = inc;
        }
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int k = 0; k < kIdxRounds; k++) {
            uint32_t before = 0, round = 0;
#pragma unroll
            for (int ww = 0; ww < kWaves; ww++) {
                const uint32_t vv = sc[ww][k];
                before += ((uint32_t)ww < w) ? vv : 0u;
                round += vv;
            }
            ex[k] += tot + before;  // newlines of the tile before this thread's bytes of round k
            tot += round;
        }
        if (tid == 0) publish_aggregate(a.status, t, tot);
        const bool staged = tot <= (uint32_t)kIdxLdsCap;
        if (staged) {
#pragma unroll
            for (int k = 0; k < kIdxRounds; k++) {
                uint32_t j = ex[k];
                const uint32_t p0 = 4096u * k + 16u * tid + 1u;  // tile offset just past byte 0 of the piece
                for (uint32_t m = m16[k]; m; m &= m - 1) pos[cur][j++] = (uint16_t)(p0 + (uint32_t)__builtin_ctz(m));
            }
        }
        if (pend) place_pending();
        if (staged) {
            pend = true;
            pt = t;
            ptot = tot;
            pb = cur;
            cur ^= 1u;
        } else {
            if (tid < 64) {
                const uint64_t e = lookback_walk(a.status, t, tot);
                if (tid == 0) sbase_sh = e;
            }
            __syncthreads();
            const uint64_t sbase = sbase_sh;
#pragma unroll
            for (int k = 0; k < kIdxRounds; k++) {
                uint64_t k1 = sbase + ex[k];
                const uint64_t x = tb + 4096u * k + 16u * tid + 1u;
                for (uint32_t m = m16[k]; m; m &= m - 1) {
                    k1++;
                    if (k1 < a.off_cap) a.off[k1] = x + (uint32_t)__builtin_ctz(m);
                }
            }
            if (t + 1 == a.ntiles) finish_last(sbase, tot);
        }
        __syncthreads();
    }
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

// Workgroups of kernel fn (256 threads, lds bytes of dynamic LDS) that fit one CU on
// the current device, at least 1; asked of the runtime once per device and kernel.
int occupancy(const void* fn, uint32_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, uint32_t>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    const auto key = std::make_tuple(dev, fn, lds);
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kWG, lds) != hipSuccess || occ < 1) occ = 1;
    cache.emplace(key, occ);
    return occ;
}

constexpr int kCompressWgPerCu = 4;  // upper bound of the persistent grid per CU (sizes the workspace)
constexpr int kDecompressWgPerCu = 4;  // upper bound of the persistent decompression grid per CU
constexpr int kIndexWgPerCu = 8;

uint32_t tiles_for(uint64_t n, uint64_t per) { return (uint32_t)((n + per - 1) / per); }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Most workgroups a plain compression of n lines launches (sizes its workspace).
size_t compress_grid_cap(uint64_t n, int cus) {
    return std::min<size_t>((size_t)cus * kCompressWgPerCu, std::max<size_t>(1, tiles_for(n, kCL)));
}


size_t ws_bytes_for(int op, uint64_t n) {
    DeviceInfo di = device_info();
    int cus = di.ok ? di.cus : 256;
    size_t h = sizeof(WsHeader);
    switch (op) {
        case ZS_OP_COMPRESS: {
            uint32_t nt = tiles_for(n, kCL);
            size_t st = ((size_t)nt * 8 + 255) & ~(size_t)255;
            size_t grid = compress_grid_cap(n, cus);
            return h + st + grid * kWG * kGenLane + grid * kCapSmall;
        }
        case ZS_OP_DECOMPRESS:
        case ZS_OP_DECOMPRESS_LINES: {
            const size_t nt = tiles_for(n, 32);  // tiles may be as small as 32 lines
            return h + align256(nt * 8);
        }
        case ZS_OP_INDEX: {
            const size_t nt = tiles_for(n, kIdxTile);
            return h + align256(nt * 8);
        }
        default:
            return 0;
    }
}


// Workspace of the binned compression, carved in this order.
struct BinnedWs {
    WsHeader* h1;      // errors, ENOSPC, the staging allocator (all launches)
    WsHeader* h2;      // the placement pass's finishing count
    BinPlan* plan;
    uint32_t* hist;    // [chunk][kMaxBins]
    uint64_t* status;  // unused (null): binned tiles take staging space from a bump allocator
    uint8_t* gen;
    uint8_t* slots;
    uint32_t* ids;
    uint32_t* pos_of;
    uint64_t* soff;    // per line in bin order: staging start << 16 | compressed length
    uint32_t* ptotal;  // placement tile totals
    uint64_t* pbase;   // their exclusive prefix, + 1
    uint8_t* staging;
    uint8_t* glines;   // line buffers of the global-memory layout, kGlStride per workgroup
    size_t bytes;
    uint32_t max_tiles, nchunks, ptiles;
};

BinnedWs binned_ws(void* ws, uint64_t n, uint64_t out_cap, int cus) {
    BinnedWs w;
    uint8_t* b = (uint8_t*)ws;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        uint8_t* p = b ? b + o : nullptr;
        o += align256(bytes);
        return p;
    };
    // every tile but the last of a bin holds at least kMinLpt lines
    w.max_tiles = (uint32_t)(n / kMinLpt + kMaxBins + 1);
    w.nchunks = tiles_for(n, kBinChunk);
    w.ptiles = tiles_for(n, kCL);
    const size_t grid = std::min<size_t>((size_t)cus * kCompressWgPerCu, w.max_tiles);
    w.h1 = (WsHeader*)take(sizeof(WsHeader));
    w.h2 = (WsHeader*)take(sizeof(WsHeader));
    w.plan = (BinPlan*)take(sizeof(BinPlan));
    w.hist = (uint32_t*)take((size_t)w.nchunks * kMaxBins * 4);
    w.status = nullptr;  // binned launches take staging space from a bump allocator, no look-back
    w.gen = take(grid * kWG * kGenLane);
    w.slots = take(grid * kCapLarge);
    w.ids = (uint32_t*)take(n * 4);
    w.pos_of = (uint32_t*)take(n * 4);
    w.soff = (uint64_t*)take((n + 1) * 8);
    w.ptotal = (uint32_t*)take((size_t)w.ptiles * 4);
    w.pbase = (uint64_t*)take(((size_t)w.ptiles + 1) * 8);
    w.staging = take(out_cap + 16);
    w.glines = take(grid * kGlStride);
    w.bytes = o;
    return w;
}

}  // namespace

// Scratch of zs_decompress_lines_noalloc, one copy per device for the life of
// the process: the workspace header and one look-back word per tile.  A set
// of at most ZS_NOALLOC_MAX_IDS requests is cut into at most 65,536 tiles of
// 256, or, when that gives fewer than two tiles per CU, into fewer than four
// tiles per CU; 69,632 words cover both on devices of up to 17,408 CUs (the
// call checks its tile count against them).
constexpr size_t kNoallocTiles = 69632;
constexpr size_t kNoallocScratchBytes = sizeof(WsHeader) + 8 * kNoallocTiles;
static_assert(ZS_NOALLOC_MAX_IDS / kDL <= kNoallocTiles, "tiles of the largest request set must fit");
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

// Device address of this device's scratch, looked up once per device (the
// array's name in host code is only a stand-in for it).  Null if the lookup
// fails.
static void* noalloc_scratch() {
    static std::mutex mu;
    static std::vector<void*> ptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    if ((int)ptr.size() <= dev) ptr.resize(dev + 1, nullptr);
    if (!ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        ptr[dev] = p;
    }
    return ptr[dev];
}

struct zs_dict {
    uint8_t* d_tables = nullptr;
    uint32_t blob_bytes = 0;
    uint32_t off_len = 0, off_exp = 0;  // LEN and EXP in the blob (the decoder stages them)
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
    d->off_len = h->off_len;
    d->off_exp = h->off_exp;
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
    const int ls = (int)compress_lds(d->comp_bytes, kCapSmall).total;
    const int lg = (int)compress_lds(d->comp_bytes, kCapGather).total_gather;
    const int ll = (int)compress_lds(d->comp_bytes, kCapLarge).total_gather;
    const int lgl = (int)compress_lds(d->comp_bytes, kCapGlobal, true).total_gather;
    if (hipFuncSetAttribute((const void*)compress_kernel<8, kCapSmall>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            ls) != hipSuccess ||
        hipFuncSetAttribute((const void*)compress_kernel<16, kCapSmall>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            ls) != hipSuccess ||
        hipFuncSetAttribute((const void*)compress_kernel<8, kCapGather>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lg) != hipSuccess ||
        hipFuncSetAttribute((const void*)compress_kernel<16, kCapGather>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lg) != hipSuccess ||
        hipFuncSetAttribute((const void*)compress_kernel<8, kCapLarge>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            ll) != hipSuccess ||
        hipFuncSetAttribute((const void*)compress_kernel<16, kCapLarge>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            ll) != hipSuccess ||
        hipFuncSetAttribute((const void*)compress_kernel_gl<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lgl) != hipSuccess ||
        hipFuncSetAttribute((const void*)compress_kernel_gl<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lgl) != hipSuccess ||
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

// One compression launch: the persistent grid of the LDS variant, at most
// max_tiles workgroups.  tab_bytes: dictionary image staged (0: none, for
// pre-processing only); lk: the parse window of the dictionary (8 or 16).
static zs_status launch_compress(uint32_t tab_bytes, uint32_t lk, const CompressArgs& a, uint32_t layout,
                                 uint32_t max_tiles, int cus, hipStream_t s, int mode = kModeCompress) {
    // plain: kCapSmall; binned: kCapGather, or for the bins that ask for it kCapLarge
    // (layout 1) or the global-memory line buffers (layout 2)
    const bool gl = layout == 2;
    const int cap = gl ? kCapGlobal : layout == 1 ? kCapLarge : (a.ids ? kCapGather : kCapSmall);
    const CompressLds cl = compress_lds(tab_bytes, cap, gl);
    const uint32_t lds = a.ids ? cl.total_gather : cl.total;
    const bool k8 = lk == 8;
    const void* kfn = mode == kModePre    ? (const void*)compress_kernel<8, kCapSmall, kModePre>
                      : mode == kModePost ? (const void*)compress_kernel<8, kCapSmall, kModePost>
                      : gl ? (k8 ? (const void*)compress_kernel_gl<8> : (const void*)compress_kernel_gl<16>)
                      : cap == kCapLarge  ? (k8 ? (const void*)compress_kernel<8, kCapLarge>
                                                : (const void*)compress_kernel<16, kCapLarge>)
                      : cap == kCapGather ? (k8 ? (const void*)compress_kernel<8, kCapGather>
                                                : (const void*)compress_kernel<16, kCapGather>)
                                          : (k8 ? (const void*)compress_kernel<8, kCapSmall>
                                                : (const void*)compress_kernel<16, kCapSmall>);
    int occ = occupancy(kfn, lds);
    if (occ > kCompressWgPerCu) occ = kCompressWgPerCu;
    uint32_t grid = (uint32_t)cus * (uint32_t)occ;
    if (grid > max_tiles) grid = max_tiles;
    if (grid < 1) grid = 1;
    void* args[] = {(void*)&a};
    if (hipLaunchKernel(kfn, dim3(grid), dim3(kWG), args, lds, s) != hipSuccess) return ZS_EDEVICE;
    return ZS_OK;
}

// Plain (one launch) compression; with d null, the ring relabelling alone
// (mode: pre- or post-processing).
// A caller's workspace: present and 256-byte aligned (the header's 64-bit
// atomics and the 16-byte accesses of the areas carved from it rely on it).
static inline bool ws_ok(const void* ws) { return ws && ((uintptr_t)ws & 255u) == 0; }

static zs_status compress_plain(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                                uint64_t n_lines, uint8_t* out, uint64_t out_cap, uint64_t* out_off, uint32_t flags,
                                void* ws, zs_result* res, hipStream_t s, int mode = kModeCompress) {
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
    uint8_t* slots = gen + compress_grid_cap(n_lines, di.cus) * kWG * kGenLane;
    if (launch_init(h, status, ntiles, (ResultOut*)res, s) != ZS_OK) return ZS_EDEVICE;
    CompressArgs a;
    a.tables = d ? d->d_tables : nullptr;
    a.tab_bytes = d ? d->comp_bytes : 0u;
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
    a.slots = slots;
    a.ids = nullptr;
    a.plan = nullptr;
    a.bin_lo = a.bin_hi = 0;
    a.ticket = nullptr;
    a.glines = nullptr;
    if (launch_compress(a.tab_bytes, d ? d->lk : 8u, a, 0, ntiles, di.cus, s, mode) != ZS_OK) return ZS_EDEVICE;
    return launch_result(h, res, s);
}

zs_status zs_compress(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                      uint64_t n_lines, uint8_t* out, uint64_t out_cap, uint64_t* out_off, uint32_t flags,
                      void* ws, size_t ws_bytes, zs_result* res, void* stream) {
    if (!d || !in_off || !out_off || !ws_ok(ws) || (!in && in_bytes)) return ZS_EINVAL;
    if (ws_bytes < zs_workspace_bytes(ZS_OP_COMPRESS, n_lines)) return ZS_EINVAL;
    if (flags & ~ZS_F_PREPROCESS) return ZS_EINVAL;
    return compress_plain(d, in, in_bytes, in_off, n_lines, out, out_cap, out_off, flags, ws, res,
                          (hipStream_t)stream);
}

zs_status zs_preprocess(const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off, uint64_t n_lines,
                        uint8_t* out, uint64_t out_cap, uint64_t* out_off, void* ws, size_t ws_bytes,
                        zs_result* res, void* stream) {
    if (!in_off || !out_off || !ws_ok(ws) || (!in && in_bytes)) return ZS_EINVAL;
    if (ws_bytes < zs_workspace_bytes(ZS_OP_COMPRESS, n_lines)) return ZS_EINVAL;
    return compress_plain(nullptr, in, in_bytes, in_off, n_lines, out, out_cap, out_off, ZS_F_PREPROCESS, ws, res,
                          (hipStream_t)stream, kModePre);
}

zs_status zs_postprocess(const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off, uint64_t n_lines,
                         uint8_t* out, uint64_t out_cap, uint64_t* out_off, void* ws, size_t ws_bytes,
                         zs_result* res, void* stream) {
    if (!in_off || !out_off || !ws_ok(ws) || (!in && in_bytes)) return ZS_EINVAL;
    if (ws_bytes < zs_workspace_bytes(ZS_OP_COMPRESS, n_lines)) return ZS_EINVAL;
    return compress_plain(nullptr, in, in_bytes, in_off, n_lines, out, out_cap, out_off, ZS_F_PREPROCESS, ws, res,
                          (hipStream_t)stream, kModePost);
}


size_t zs_binned_workspace_bytes(uint64_t n_lines, uint64_t out_cap) {
    DeviceInfo di = device_info();
    return binned_ws(nullptr, n_lines, out_cap, di.ok ? di.cus : 256).bytes;
}

zs_status zs_compress_binned(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                             uint64_t n_lines, uint8_t* out, uint64_t out_cap, uint64_t* out_off, uint32_t flags,
                             const zs_bin_config* cfg, void* ws, size_t ws_bytes, zs_result* res, void* stream) {
    if (!d || !in_off || !out_off || !ws_ok(ws) || !cfg || (!in && in_bytes)) return ZS_EINVAL;
    if (flags & ~ZS_F_PREPROCESS) return ZS_EINVAL;
    if (n_lines >= (1ull << 32)) return ZS_EINVAL;
    const uint32_t nb = cfg->nbins;
    if (nb < 1 || nb > kMaxBins) return ZS_EINVAL;
    for (uint32_t i = 0; i + 1 < nb; i++)
        if (cfg->edges[i] == 0 || (i > 0 && cfg->edges[i] <= cfg->edges[i - 1])) return ZS_EINVAL;
    for (uint32_t i = 0; i < nb; i++)
        if (cfg->lines_per_tile[i] < kMinLpt || cfg->lines_per_tile[i] > (uint32_t)kCL || cfg->large_lds[i] > 2)
            return ZS_EINVAL;
    DeviceInfo di = device_info();
    if (!di.ok) return ZS_EDEVICE;
    const uint64_t cap = out ? out_cap : 0;
    BinnedWs w = binned_ws(ws, n_lines, cap, di.cus);
    if (ws_bytes < w.bytes) return ZS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (n_lines == 0) {
        hipLaunchKernelGGL(empty_result_kernel, dim3(1), dim3(1), 0, s, out_off, (ResultOut*)res);
        return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
    }
    // processing order: longest bin first
    BinInit bi;
    memset(&bi, 0, sizeof bi);
    bi.nbins = nb;
    uint32_t large[kMaxBins] = {0};
    for (uint32_t b = 0; b < nb; b++) {
        const uint32_t i = nb - 1 - b;  // the configuration's bin
        bi.upper[b] = (i == nb - 1) ? 0xFFFFFFFFu : cfg->edges[i];
        bi.lpt[b] = cfg->lines_per_tile[i];
        large[b] = cfg->large_lds[i];
    }
    hipLaunchKernelGGL(binned_init_kernel, dim3(1), dim3(64), 0, s, w.h1, w.h2, w.plan, bi, (ResultOut*)res);
    BinArgs ba;
    ba.in_off = in_off;
    ba.n = n_lines;
    ba.in_bytes = in_bytes;
    ba.plan = w.plan;
    ba.hist = w.hist;
    ba.nchunks = w.nchunks;
    ba.ids = w.ids;
    ba.pos_of = w.pos_of;
    const uint32_t bgrid = w.nchunks;  // one workgroup per chunk
    hipLaunchKernelGGL(bin_count_kernel, dim3(bgrid), dim3(kWG), 0, s, ba);
    hipLaunchKernelGGL(bin_plan_kernel, dim3(1), dim3(kWG), 0, s, ba);
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(bgrid), dim3(kWG), 0, s, ba);
    if (hipGetLastError() != hipSuccess) return ZS_EDEVICE;
    // one compression launch per run of bins that share an LDS layout
    CompressArgs a;
    a.tables = d->d_tables;
    a.tab_bytes = d->comp_bytes;
    a.in = in;
    a.in_bytes = in_bytes;
    a.in_off = in_off;
    a.n = n_lines;
    a.out = out ? w.staging : nullptr;
    a.out_cap = out ? out_cap : ~0ull;
    a.out_off = w.soff;
    a.flags = flags;
    a.ntiles = 0;
    a.ws = w.h1;
    a.status = w.status;
    a.gen = w.gen;
    a.slots = w.slots;
    a.ids = w.ids;
    a.plan = w.plan;
    a.glines = w.glines;
    uint32_t b = 0, launch = 0;
    while (b < nb) {
        uint32_t e = b + 1;
        while (e < nb && large[e] == large[b]) e++;
        a.bin_lo = b;
        a.bin_hi = e;
        a.ticket = (uint32_t*)((uint8_t*)w.plan + offsetof(BinPlan, ticket)) + launch;
        // an upper bound of this launch's tiles sizes the grid
        uint64_t most = 0;
        for (uint32_t k = b; k < e; k++) most += (n_lines + bi.lpt[k] - 1) / bi.lpt[k];
        if (launch_compress(d->comp_bytes, d->lk, a, large[b], (uint32_t)std::min<uint64_t>(most, w.max_tiles),
                            di.cus, s) != ZS_OK)
            return ZS_EDEVICE;
        b = e;
        launch++;
    }
    // back to input order
    PlaceArgs pa;
    pa.pos_of = w.pos_of;
    pa.soff = w.soff;
    pa.staging = w.staging;
    pa.staging_bytes = cap + 16;  // binned_ws: the staging area holds the output's capacity + 16
    pa.n = n_lines;
    pa.out = out;
    pa.out_cap = out ? out_cap : ~0ull;
    pa.out_off = out_off;
    pa.ntiles = w.ptiles;
    pa.tile_total = w.ptotal;
    pa.tile_base = w.pbase;
    pa.ws = w.h1;
    const uint32_t pgrid = std::min(w.ptiles, (uint32_t)di.cus * 8);
    hipLaunchKernelGGL(place_count_kernel, dim3(pgrid), dim3(kWG), 0, s, pa);
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(kScanWG), 0, s, w.ptotal, w.pbase, w.ptiles);
    // one workgroup per tile: the hardware starts the next tile's workgroup as soon
    // as a slot frees (11% faster than a grid-stride loop over 8 workgroups per CU)
    hipLaunchKernelGGL(place_write_kernel, dim3(w.ptiles), dim3(kWG), 0, s, pa);
    return launch_result(w.h1, res, s);
}


zs_status zs_autotune_binned(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                             uint64_t n_lines, uint32_t flags, zs_bin_config* best, double* best_ms,
                             double* plain_ms, uint32_t* n_tried, void* stream) {
    if (!d || !in_off || !best || n_lines == 0 || (!in && in_bytes)) return ZS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // line lengths on the host: their quantiles give the candidate edges
    std::vector<uint64_t> off(n_lines + 1);
    if (hipMemcpyAsync(off.data(), in_off, off.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ZS_EDEVICE;
    std::vector<uint32_t> len(n_lines);
    for (uint64_t k = 0; k < n_lines; k++)
        len[k] = (uint32_t)std::min<uint64_t>(off[k + 1] > off[k] ? off[k + 1] - off[k] - 1 : 0, 1u << 20);
    std::sort(len.begin(), len.end());
    auto q = [&](double f) {
        uint32_t v = len[std::min<uint64_t>(n_lines - 1, (uint64_t)(f * (double)n_lines))];
        return std::max(8u, (v + 7) & ~7u);
    };
    const uint32_t lmax = len.back();
    // buffers for the trials (exact output size from a size-only pass)
    uint8_t *out = nullptr, *ws = nullptr, *wsb = nullptr;
    uint64_t* oo = nullptr;
    zs_result* res = nullptr;
    zs_status rc = ZS_OK;
    const size_t wsp = zs_workspace_bytes(ZS_OP_COMPRESS, n_lines);
    if (hipMalloc(&oo, (n_lines + 1) * 8) != hipSuccess || hipMalloc(&ws, wsp) != hipSuccess ||
        hipMalloc(&res, sizeof(zs_result)) != hipSuccess) {
        rc = ZS_ENOMEM;
    }
    uint64_t total = 0;
    if (rc == ZS_OK) rc = zs_compress(d, in, in_bytes, in_off, n_lines, nullptr, 0, oo, flags, ws, wsp, res, s);
    if (rc == ZS_OK && (hipMemcpyAsync(&total, oo + n_lines, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
        rc = ZS_EDEVICE;
    const size_t wsbytes = zs_binned_workspace_bytes(n_lines, total);
    if (rc == ZS_OK && (hipMalloc(&out, total + 16) != hipSuccess || hipMalloc(&wsb, wsbytes) != hipSuccess))
        rc = ZS_ENOMEM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == ZS_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = ZS_EDEVICE;
    // time one configuration (null: plain zs_compress): one warm-up, best of 3
    auto run = [&](const zs_bin_config* c, double* ms) -> zs_status {
        double bestt = 1e30;
        for (int r = 0; r < 4; r++) {
            if (hipEventRecord(e0, s) != hipSuccess) return ZS_EDEVICE;
            zs_status z = c ? zs_compress_binned(d, in, in_bytes, in_off, n_lines, out, total + 16, oo, flags, c, wsb,
                                                 wsbytes, res, s)
                            : zs_compress(d, in, in_bytes, in_off, n_lines, out, total + 16, oo, flags, ws, wsp, res, s);
            if (z != ZS_OK) return z;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ZS_EDEVICE;
            float t = 0;
            if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return ZS_EDEVICE;
            if (r > 0) bestt = std::min(bestt, (double)t);
        }
        *ms = bestt;
        return ZS_OK;
    };
    double tplain = 0;
    if (rc == ZS_OK) rc = run(nullptr, &tplain);
    // candidates: edge sets x lines per tile of the longest bin x its LDS layout
    std::vector<std::vector<uint32_t>> edge_sets = {{},
                                                    {q(0.90)},
                                                    {q(0.75)},
                                                    {q(0.95)},
                                                    {128},
                                                    {192},
                                                    {256},
                                                    {q(0.50), q(0.90)},
                                                    {q(0.75), q(0.95)},
                                                    {128, 512},
                                                    {q(0.90), 512}};
    double tbest = 1e30;
    zs_bin_config cbest;
    memset(&cbest, 0, sizeof cbest);
    uint32_t tried = 0;
    for (auto& es : edge_sets) {
        std::vector<uint32_t> e;
        for (uint32_t v : es)
            if (v < lmax && (e.empty() || v > e.back())) e.push_back(v);
        if (e.size() != es.size() && !es.empty()) continue;  // a degenerate set repeats a smaller one
        const uint32_t nb = (uint32_t)e.size() + 1;
        for (uint32_t lpt : {256u, 128u, 64u, 32u}) {
            for (uint32_t lg : {0u, 1u, 2u}) {
                if (nb == 1 && lpt != 256) continue;
                zs_bin_config c;
                memset(&c, 0, sizeof c);
                c.nbins = nb;
                for (uint32_t i = 0; i + 1 < nb; i++) c.edges[i] = e[i];
                for (uint32_t i = 0; i < nb; i++) c.lines_per_tile[i] = 256;
                c.lines_per_tile[nb - 1] = lpt;
                c.large_lds[nb - 1] = lg;
                double t = 0;
                if (rc == ZS_OK) rc = run(&c, &t);
                if (rc != ZS_OK) break;
                tried++;
                if (t < tbest) {
                    tbest = t;
                    cbest = c;
                }
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (ws) (void)hipFree(ws);
    if (wsb) (void)hipFree(wsb);
    if (oo) (void)hipFree(oo);
    if (res) (void)hipFree(res);
    if (rc != ZS_OK) return rc;
    *best = cbest;
    if (best_ms) *best_ms = tbest;
    if (plain_ms) *plain_ms = tplain;
    if (n_tried) *n_tried = tried;
    return ZS_OK;
}

struct zs_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

zs_status zs_graph_begin(void* stream) {
    if (!stream) return ZS_EINVAL;
    return hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal) == hipSuccess ? ZS_OK
                                                                                                    : ZS_EDEVICE;
}

zs_status zs_graph_end(void* stream, zs_graph** out) {
    if (!stream || !out) return ZS_EINVAL;
    zs_graph* g = new (std::nothrow) zs_graph;
    if (!g) return ZS_ENOMEM;
    if (hipStreamEndCapture((hipStream_t)stream, &g->graph) != hipSuccess || !g->graph) {
        delete g;
        return ZS_EDEVICE;
    }
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        return ZS_EDEVICE;
    }
    *out = g;
    return ZS_OK;
}

zs_status zs_graph_launch(zs_graph* g, void* stream) {
    if (!g) return ZS_EINVAL;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? ZS_OK : ZS_EDEVICE;
}

void zs_graph_destroy(zs_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

// Requests per tile of a decompression of nreq lines or ids: small request sets
// are cut into smaller tiles so that more workgroups share them.
static uint32_t decompress_tile_lines(uint64_t nreq, int cus) {
    const uint64_t want = (uint64_t)cus * 2;
    uint32_t tl = kDL;
    while (tl > 32 && (nreq + tl - 1) / tl < want) tl >>= 1;
    return tl;
}

// ws_bytes is checked against zs_workspace_bytes(op, nreq) when exact_ws is
// false, else against what this call's tiles need (the scratch of the
// allocation-free entry point).
static zs_status decompress_common(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                                   uint64_t n_lines, const uint64_t* ids, uint64_t nreq, uint8_t* out,
                                   uint64_t out_cap, uint64_t* out_off, void* ws, size_t ws_bytes, zs_result* res,
                                   void* stream, int op, bool exact_ws = false) {
    if (!d || !in_off || !out_off || !ws_ok(ws) || (!in && in_bytes)) return ZS_EINVAL;
    if (!exact_ws && ws_bytes < zs_workspace_bytes(op, nreq)) return ZS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (nreq == 0) {
        hipLaunchKernelGGL(empty_result_kernel, dim3(1), dim3(1), 0, s, out_off, (ResultOut*)res);
        return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
    }
    DeviceInfo di = device_info();
    if (!di.ok) return ZS_EDEVICE;
    const uint32_t tl = decompress_tile_lines(nreq, di.cus);
    const uint32_t ntiles = tiles_for(nreq, tl);
    if (exact_ws && ws_bytes < sizeof(WsHeader) + (size_t)ntiles * 8) return ZS_EINVAL;
    WsHeader* h = (WsHeader*)ws;
    uint64_t* status = (uint64_t*)(h + 1);
    if (launch_init(h, status, ntiles, (ResultOut*)res, s) != ZS_OK) return ZS_EDEVICE;
    DecompressArgs a;
    a.tl = tl;
    a.tables = d->d_tables;
    a.off_len = d->off_len;
    a.off_exp = d->off_exp;
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
    const uint32_t lds = decompress_lds().total;
    int occ = occupancy((const void*)decompress_kernel, lds);
    if (occ > kDecompressWgPerCu) occ = kDecompressWgPerCu;
    uint32_t grid = (uint32_t)di.cus * (uint32_t)occ;
    if (grid > ntiles) grid = ntiles;
    hipLaunchKernelGGL(decompress_kernel, dim3(grid), dim3(kWG), lds, s, a);
    return launch_result(h, res, s);
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

zs_status zs_decompress_lines_noalloc(const zs_dict* d, const uint8_t* in, uint64_t in_bytes,
                                      const uint64_t* in_off, uint64_t n_lines, const uint64_t* ids, uint64_t n_ids,
                                      uint8_t* out, uint64_t out_cap, uint64_t* out_off, zs_result* res,
                                      void* stream) {
    if (n_ids && !ids) return ZS_EINVAL;
    if (n_ids > ZS_NOALLOC_MAX_IDS) return ZS_EINVAL;
    void* ws = noalloc_scratch();
    if (!ws) return ZS_EDEVICE;
    return decompress_common(d, in, in_bytes, in_off, n_lines, ids, n_ids, out, out_cap, out_off, ws,
                             kNoallocScratchBytes, res, stream, ZS_OP_DECOMPRESS_LINES, true);
}

zs_status zs_index_lines(const uint8_t* buf, uint64_t len, uint64_t* off, uint64_t off_cap, uint64_t* n_lines_out,
                         void* ws, size_t ws_bytes, zs_result* res, void* stream) {
    if ((!buf && len) || !n_lines_out || !ws_ok(ws) || (!off && off_cap)) return ZS_EINVAL;
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
    int occ = occupancy((const void*)index_kernel, 0);
    if (occ > kIndexWgPerCu) occ = kIndexWgPerCu;
    uint32_t grid = (uint32_t)di.cus * (uint32_t)occ;
    if (grid > ntiles) grid = ntiles;
    hipLaunchKernelGGL(index_kernel, dim3(grid), dim3(kWG), 0, s, a);
    return launch_result(h, res, s);
}

}  // extern "C"
