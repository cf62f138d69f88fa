// zs_tables.hpp - layout of the compiled dictionary image shared by the host
// compiler (zs_dict.cpp) and the kernels (zs_kernels.hip).
//
// The image is one contiguous blob, uploaded once per dictionary and staged
// into LDS by every workgroup.  Sections, in this order, each 16-byte aligned:
//
//   header               TableHeader
//   LEN  [256]      u8   expansion length of each code byte (0 = not a code)
//   COL  [256]      u8   byte -> column of the match automaton
//   CODE1[256]      u8   byte -> code whose expansion is that single byte (0 = none)
//   TRANS[S][C]     u16  automaton transition, state x column -> state
//   OUTK [S][LK]    i8   per state and length L = 1..LK: the low bits of the DP
//                        key when a pattern of length L starts here (31 - L),
//                        or -1 when none does (sign-extended, it disables the
//                        length in the key's OR: 0xFFFFFFFF)
//   CODE [S][LK]    u8   per state and length L >= 2: the code of that pattern
//   EXP  [256][16]  u8   expansion bytes (decoder table, Sec. IV-D-2)
//
// The compressor stages [0, off_exp) in LDS, the decoder the header, LEN and
// EXP.
//
// The automaton recognises every dictionary pattern that STARTS at the
// current position while the line is read from its end backwards: it is the
// Aho-Corasick automaton of the reversed patterns run over the reversed line,
// so its outputs at position i are exactly the lengths L with s[i..i+L) in
// the dictionary - the edges of the graph G of Sec. IV-D-1 that leave node i.
// Characters that occur only as one-character codes share column 1, whose
// transition from every state is the fixed state 1 (output {1}, transitions
// equal to the root's); characters in no pattern share column 0, which leads
// to the root (state 0, no output).
#pragma once
#include <stdint.h>

namespace zs {

constexpr int kExpStride = 16;  // bytes per EXP row
constexpr int kMaxStates = 4096;
constexpr int kMaxTransBytes = 32768;

struct TableHeader {
    uint32_t lmax;     // longest expansion
    uint32_t lk;       // lengths tracked by the DP window: 8 or 16
    uint32_t nstates;  // S
    uint32_t ncols;    // C
    uint32_t off_len, off_col, off_code1, off_trans, off_outk, off_code, off_exp;
    uint32_t blob_bytes;  // total image size, header included
    uint32_t ncodes;
    uint32_t pad[3];
};
static_assert(sizeof(TableHeader) == 64, "header is 64 bytes");

constexpr uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

}  // namespace zs
