// zs_common.hpp - device-side building blocks shared by the kernels: block
// scans for wave64 workgroups, the single-pass decoupled look-back scan across
// tiles, the workspace header and the result finaliser.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zs {

constexpr int kWG = 256;  // threads per workgroup in every kernel
constexpr int kWaves = kWG / 64;

// Workspace header, at the start of the caller's workspace.  Zeroed by the
// init kernel of every call.
struct WsHeader {
    uint32_t ticket;   // next tile to claim
    uint32_t done;     // unused (cleared with the header)
    uint32_t enospc;   // set when the output does not fit
    uint32_t pad0;
    uint64_t errkey;   // min over bad lines of (index << 3 | error kind); ~0 = none
    uint64_t total;    // total output bytes (or lines, for the index)
    uint64_t alloc;    // binned compression: staging bytes handed out so far
    uint64_t pad[3];
};
static_assert(sizeof(WsHeader) == 64, "64-byte header");

// Error kinds carried in the low 3 bits of errkey.
constexpr uint32_t kErrInval = 1, kErrCorrupt = 2;

__device__ inline void note_error(WsHeader* h, uint64_t index, uint32_t kind) {
    atomicMin((unsigned long long*)&h->errkey, (unsigned long long)((index << 3) | kind));
}

// ---- decoupled look-back (Merrill & Garland, "Single-pass Parallel Prefix Scan
//      with Decoupled Look-back", 2016).  One 64-bit word per tile: the top two
//      bits say what the low 62 hold (1 = this tile's aggregate, 2 = inclusive
//      prefix through this tile).
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagInc = 2ull << 62, kValMask = (1ull << 62) - 1;

// The words carry sizes only: no workgroup reads data another one wrote, so
// no acquire/release ordering is needed (at device scope it would write back
// and invalidate the XCD's L2 at every access).  The words themselves are read
// and written with read-modify-write atomics, which are performed at the
// device's coherence point: a plain load, even a device-scope one, may be
// served from a copy in the reading XCD's own L2 and miss another XCD's update.
__device__ inline void status_store(uint64_t* p, uint64_t v) {
    (void)__hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t status_load(uint64_t* p) {
    return __hip_atomic_fetch_add(p, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Publish a tile's aggregate (tile 0 publishes its inclusive prefix at once).
// Called by one lane.
__device__ inline void publish_aggregate(uint64_t* status, uint32_t t, uint64_t agg) {
    status_store(&status[t], (t == 0 ? kFlagInc : kFlagAgg) | agg);
}

// Called by all 64 lanes of one wave of the workgroup owning tile t, whose
// aggregate is already published.  Returns (in every lane) the exclusive
// prefix, the sum of all tiles before t, and publishes t's inclusive prefix.
// Each round reads the status words of the 64 closest unvisited predecessors
// at once: the nearest one holding an inclusive prefix ends the walk, the
// aggregates in front of it are added; a round in which a nearer predecessor
// has not published yet is read again.
__device__ inline uint64_t lookback_walk(uint64_t* status, uint32_t t, uint64_t agg) {
    const int lane = threadIdx.x & 63;
    if (t == 0) return 0;
    uint64_t excl = 0;
    int64_t top = (int64_t)t - 1;
    while (true) {
        const int64_t j = top - lane;
        const uint64_t s = (j >= 0) ? status_load(&status[j]) : kFlagInc;
        const uint64_t f = s & ~kValMask;
        const uint64_t inc = __ballot(f == kFlagInc);
        const uint64_t notready = __ballot(f == 0);
        const int first = inc ? __builtin_ctzll(inc) : 64;
        const uint64_t before = first >= 64 ? ~0ull : ((1ull << first) | ((1ull << first) - 1));
        if (notready & before) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum64((uint64_t)lane <= (uint64_t)first ? (s & kValMask) : 0ull);
        if (first < 64) break;
        top -= 64;
    }
    if (lane == 0) status_store(&status[t], kFlagInc | (excl + agg));
    return excl;
}

// Publish and walk in one go.
__device__ inline uint64_t lookback(uint64_t* status, uint32_t t, uint64_t agg) {
    if ((threadIdx.x & 63) == 0) publish_aggregate(status, t, agg);
    return lookback_walk(status, t, agg);
}

// ---- scans over one workgroup of kWG threads (wave64)
// Inclusive scan over the 64 lanes (all lanes active): DPP row shifts inside
// each row of 16 lanes, then the totals of the rows before, read from lanes
// 15, 31 and 47.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
    const uint32_t t0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t t1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t t2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    const uint32_t row = (threadIdx.x & 63) >> 4;
    v += (row >= 1 ? t0 : 0u) + (row >= 2 ? t1 : 0u) + (row >= 3 ? t2 : 0u);
    return v;
}

// Exclusive scan of v over the workgroup; *total receives the sum.
// scratch: kWaves + 1 uint32 in LDS.  Contains barriers: call uniformly.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* scratch, uint32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) scratch[w] = inc;
    __syncthreads();
    uint32_t base = 0, sum = 0;
#pragma unroll
    for (int k = 0; k < kWaves; k++) {
        uint32_t s = scratch[k];
        base += (k < w) ? s : 0;
        sum += s;
    }
    __syncthreads();
    *total = sum;
    return base + inc - v;
}

// Same for 64-bit values.
__device__ inline uint64_t wave_incl_scan64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

__device__ inline uint64_t block_excl_scan64(uint64_t v, uint64_t* scratch, uint64_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t inc = wave_incl_scan64(v);
    if (lane == 63) scratch[w] = inc;
    __syncthreads();
    uint64_t base = 0, sum = 0;
#pragma unroll
    for (int k = 0; k < kWaves; k++) {
        uint64_t s = scratch[k];
        base += (k < w) ? s : 0;
        sum += s;
    }
    __syncthreads();
    *total = sum;
    return base + inc - v;
}

// Claim the next tile: one atomic per workgroup, broadcast through LDS.
__device__ inline uint32_t claim_tile(WsHeader* h, uint32_t* s_slot) {
    if (threadIdx.x == 0) *s_slot = atomicAdd(&h->ticket, 1u);
    __syncthreads();
    uint32_t t = *s_slot;
    __syncthreads();
    return t;
}

// The caller's result word (zs_result), written after a call's last kernel.
struct ResultOut {
    int32_t code;
    int32_t reserved;
    int64_t first_bad;
};

// The call's result from the error words of header h: the first bad line's
// error, else ENOSPC, else success.
__device__ inline void write_result(WsHeader* h, ResultOut* res) {
    uint64_t ek = __hip_atomic_load(&h->errkey, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t nospc = __hip_atomic_load(&h->enospc, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    int32_t code = 0;
    int64_t fb = -1;
    if (ek != ~0ull) {
        fb = (int64_t)(ek >> 3);
        code = ((ek & 7) == kErrInval) ? -1 : -3;
    } else if (nospc) {
        code = -2;
    }
    res->code = code;
    res->reserved = 0;
    res->first_bad = fb;
}

// Copy bytes [glo, ghi) of an output stream from an LDS stage whose byte 0
// corresponds to the global address a0 (a0 is 16-byte aligned, a0 <= glo).
// Whole 16-byte chunks are written with one store, the two partial chunks at
// the ends byte by byte, so neighbouring tiles' bytes are never touched.
__device__ inline void flush_stage(uint8_t* out, uint64_t glo, uint64_t ghi, uintptr_t a0, const uint8_t* stage) {
    if (ghi <= glo) return;
    uintptr_t lo = (uintptr_t)(out + glo), hi = (uintptr_t)(out + ghi);
    uintptr_t nchunks = (hi - a0 + 15) >> 4;
    for (uintptr_t c = threadIdx.x; c < nchunks; c += kWG) {
        uintptr_t ca = a0 + (c << 4);
        const uint8_t* src = stage + (c << 4);
        if (ca >= lo && ca + 16 <= hi) {
            *(uint4*)ca = *(const uint4*)src;
        } else {
            for (int k = 0; k < 16; k++) {
                uintptr_t p = ca + k;
                if (p >= lo && p < hi) *(uint8_t*)p = src[k];
            }
        }
    }
}

// Load global bytes [lo, hi) of `src` into an LDS buffer whose byte 0
// corresponds to the 16-byte aligned address a0 <= src+lo.  Chunks that lie
// fully inside [src, src+limit) are read with 16-byte loads; chunks that would
// cross either end of the buffer are read byte by byte.
__device__ inline void load_range(const uint8_t* src, uint64_t limit, uint64_t lo, uint64_t hi, uintptr_t a0,
                                  uint8_t* dst) {
    if (hi <= lo) return;
    uintptr_t blo = (uintptr_t)src, bhi = (uintptr_t)(src + limit);
    uintptr_t rlo = (uintptr_t)(src + lo), rhi = (uintptr_t)(src + hi);
    uintptr_t nchunks = (rhi - a0 + 15) >> 4;
    for (uintptr_t c = threadIdx.x; c < nchunks; c += kWG) {
        uintptr_t ca = a0 + (c << 4);
        uint8_t* d = dst + (c << 4);
        if (ca >= blo && ca + 16 <= bhi) {
            *(uint4*)d = *(const uint4*)ca;
        } else {
            for (int k = 0; k < 16; k++) {
                uintptr_t p = ca + k;
                d[k] = (p >= blo && p < bhi && p >= rlo && p < rhi) ? *(const uint8_t*)p : (uint8_t)0;
            }
        }
    }
}

// Per 4-byte word: bit 7 of each byte set where the byte equals the same byte
// of pat (exact: no carries cross bytes).
__device__ inline uint32_t swar_eq_bytes(uint32_t w, uint32_t pat) {
    const uint32_t x = w ^ pat;
    return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
}

// LDS stage writer of one thread: appends its bytes in order from stage index
// s0.  Whole dwords that hold only this thread's bytes are written as dwords,
// the partial ones at the two ends byte by byte (the neighbouring threads
// write the rest of them).
struct StageWriter {
    uint8_t* stage;
    uint32_t s0, s, a;
    uint64_t acc;  // bytes [a, s) not yet written; s - a < 4 between calls
    __device__ __forceinline__ void begin(uint8_t* st, uint32_t at) {
        stage = st;
        s0 = s = at;
        a = at & ~3u;
        acc = 0;
    }
    __device__ __forceinline__ void put_dword(uint32_t at, uint32_t v) {
        if (at >= s0) {
            *(uint32_t*)(stage + at) = v;
        } else {
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (at + j >= s0) stage[at + j] = (uint8_t)(v >> (8 * j));
        }
    }
    // m (1..4) bytes: the low bytes of v, its other bytes zero
    __device__ __forceinline__ void add(uint32_t v, uint32_t m) {
        acc |= (uint64_t)v << (8 * (s - a));
        s += m;
        if (s - a >= 4) {
            put_dword(a, (uint32_t)acc);
            acc >>= 32;
            a += 4;
        }
    }
    __device__ __forceinline__ void finish() {
        for (uint32_t x = a; x < s; x++)
            if (x >= s0) stage[x] = (uint8_t)(acc >> (8 * (x - a)));
    }
};

// Bytes [lo, hi) (clamped to 0..4) of a dword as a mask.
__device__ inline uint32_t dword_byte_mask(int32_t lo, int32_t hi) {
    lo = max(lo, 0);
    hi = min(hi, 4);
    if (hi <= lo) return 0u;
    const uint32_t up = hi == 4 ? 0xFFFFFFFFu : ((1u << (8 * hi)) - 1u);
    return up & ~((1u << (8 * lo)) - 1u);
}

// OR into the 16-byte piece w its bytes [k0, k1) (0 <= k0 < k1 <= 16), taken from
// the bytes at address sa onwards (piece byte k0 is the byte at sa): two aligned
// 16-byte loads from sa's 16-byte boundary, shifted into place.  The caller checks
// that both loads lie inside the buffer.
__device__ inline void or_shifted_piece(uint32_t w[4], uintptr_t sa, uint32_t k0, uint32_t k1) {
    const uintptr_t c0 = sa & ~(uintptr_t)15;
    const uint4 x = *(const uint4*)c0, y = *(const uint4*)(c0 + 16);
    // piece byte k is byte k + e of 16 zero bytes, then x, then y
    const uint32_t e = (uint32_t)(sa - c0) + 16u - k0;
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
    for (int j = 0; j < 4; j++)
        w[j] |= __builtin_amdgcn_alignbyte(d[j + 1], d[j], rb) &
                dword_byte_mask((int32_t)k0 - 4 * j, (int32_t)k1 - 4 * j);
}

// Copy total bytes from a 16-byte aligned buffer (a tile parked in its global
// slot, or a stage in LDS) to out[base, base + total) directly: each thread
// loads the two source chunks that one 16-byte chunk of the destination
// straddles, shifts them into place and stores 16 bytes (byte stores at the
// two partial ends).  No source chunk past the one holding byte total - 1 is
// read.
__device__ inline void copy_slot_direct(uint8_t* out, const uint8_t* slot, uint32_t total, uint64_t base) {
    const uintptr_t dst = (uintptr_t)(out + base);
    const uintptr_t a0 = dst & ~(uintptr_t)15;
    const int32_t lead = (int32_t)(dst - a0);
    const uint32_t nch = ((uint32_t)lead + total + 15) >> 4;
    const uint4* s16 = (const uint4*)slot;
    for (uint32_t c = threadIdx.x; c < nch; c += kWG) {
        const int32_t sb = (int32_t)(c * 16) - lead;  // slot byte of the chunk's first byte
        const int32_t i0 = sb >> 4;                   // arithmetic: -1 for the first chunk when lead > 0
        const uint32_t sh = (uint32_t)sb & 15u;
        const uint4 A = i0 >= 0 ? s16[i0] : make_uint4(0, 0, 0, 0);
        const uint4 B = (uint32_t)(i0 + 1) * 16u < total ? s16[i0 + 1] : make_uint4(0, 0, 0, 0);
        const uint32_t w[8] = {A.x, A.y, A.z, A.w, B.x, B.y, B.z, B.w};
        const uint32_t q = sh >> 2, r = sh & 3u;
        uint32_t d[5];
#pragma unroll
        for (int j = 0; j < 5; j++) d[j] = q == 0 ? w[j] : q == 1 ? w[j + 1] : q == 2 ? w[j + 2] : w[j + 3];
        uint32_t o[4];
#pragma unroll
        for (int j = 0; j < 4; j++) o[j] = __builtin_amdgcn_alignbyte(d[j + 1], d[j], r);
        uint8_t* p = (uint8_t*)(a0 + ((uintptr_t)c << 4));
        if (sb >= 0 && sb + 16 <= (int32_t)total) {
            *(uint4*)p = make_uint4(o[0], o[1], o[2], o[3]);
        } else {
#pragma unroll
            for (int k = 0; k < 16; k++)
                if (sb + k >= 0 && sb + k < (int32_t)total) p[k] = (uint8_t)(o[k >> 2] >> (8 * (k & 3)));
        }
    }
}

}  // namespace zs
