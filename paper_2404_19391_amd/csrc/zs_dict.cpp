// zs_dict.cpp - host side of the dictionary: validation and compilation of the
// code table into the image the kernels stage in LDS (layout in zs_tables.hpp).
// Pure C++, no HIP calls, so it also runs where no GPU is present.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "zs_tables.hpp"
#include "../../include/zsmiles.h"

namespace {

bool is_code_byte(int b) { return (b >= 0x21 && b <= 0x7E) || (b >= 0xA1 && b <= 0xFF); }

struct Trie {
    // children per column; -1 = none
    std::vector<std::vector<int>> child;
    std::vector<int> depth;
    std::vector<int> term_code;  // code ending here (pattern reversed), -1 = none
    std::vector<std::vector<uint8_t>> str;  // the reversed-pattern prefix spelt by the node
    int ncols;
    explicit Trie(int c) : ncols(c) {}
    int add(int d) {
        child.emplace_back(ncols, -1);
        depth.push_back(d);
        term_code.push_back(-1);
        str.emplace_back();
        return (int)child.size() - 1;
    }
};

}  // namespace

// Validate and compile.  Returns ZS_OK and fills `blob`, or ZS_EINVAL.
extern "C" int zsi_compile_dict(const uint8_t* len, const uint8_t* exp, std::vector<uint8_t>* blob_out);

int zsi_compile_dict(const uint8_t* len, const uint8_t* exp, std::vector<uint8_t>* blob_out) {
    using namespace zs;
    // ---- validation (Sec. IV-B: printable codes; space escapes, newline separates)
    int lmax = 0, ncodes = 0;
    std::map<std::string, int> seen;
    for (int b = 0; b < 256; b++) {
        int L = len[b];
        if (!L) continue;
        if (!is_code_byte(b) || L > (int)ZS_LMAX_CAP) return ZS_EINVAL;
        std::string e((const char*)exp + b * kExpStride, (size_t)L);
        for (unsigned char c : e)
            if (c < 0x21 || c > 0x7E) return ZS_EINVAL;
        if (!seen.emplace(e, b).second) return ZS_EINVAL;
        lmax = std::max(lmax, L);
        ncodes++;
    }
    const int lk = lmax <= 8 ? 8 : 16;

    // ---- columns: 0 = in no pattern, 1 = only as a one-byte pattern, 2.. = in a longer pattern
    std::vector<int> col(256, 0);
    std::vector<uint8_t> code1(256, 0);
    bool in_multi[256] = {false};
    for (auto& kv : seen)
        if (kv.first.size() >= 2)
            for (unsigned char c : kv.first) in_multi[c] = true;
    int ncols = 2;
    for (int c = 0; c < 256; c++)
        if (in_multi[c]) col[c] = ncols++;
    for (auto& kv : seen)
        if (kv.first.size() == 1) {
            unsigned char c = (unsigned char)kv.first[0];
            code1[c] = (uint8_t)kv.second;
            if (!in_multi[c]) col[c] = 1;
        }

    // ---- trie of the reversed patterns over columns >= 2 (node 0 root, node 1 the
    //      shared "one-byte-only" state)
    Trie t(ncols);
    t.add(0);
    t.add(1);
    for (auto& kv : seen) {
        const std::string& p = kv.first;
        if (p.size() == 1 && !in_multi[(unsigned char)p[0]]) continue;
        int u = 0;
        for (int k = (int)p.size() - 1; k >= 0; k--) {
            unsigned char c = (unsigned char)p[k];
            int cc = col[c];
            if (t.child[u][cc] < 0) {
                int v = t.add(t.depth[u] + 1);
                t.str[v] = t.str[u];
                t.str[v].push_back(c);
                t.child[u][cc] = v;
            }
            u = t.child[u][cc];
            if ((int)t.child.size() > kMaxStates) return ZS_EINVAL;
        }
        t.term_code[u] = kv.second;
    }
    const int S = (int)t.child.size();
    if ((size_t)S * (size_t)ncols * 2 > (size_t)kMaxTransBytes) return ZS_EINVAL;

    // ---- failure links and the full transition function (breadth first)
    std::vector<int> fail(S, 0);
    std::vector<std::vector<int>> delta(S, std::vector<int>(ncols, 0));
    for (int s = 0; s < S; s++) {
        delta[s][0] = 0;
        delta[s][1] = 1;
    }
    std::deque<int> q;
    for (int c = 2; c < ncols; c++) {
        int v = t.child[0][c];
        if (v >= 0) {
            fail[v] = 0;
            delta[0][c] = v;
            q.push_back(v);
        } else {
            delta[0][c] = 0;
        }
    }
    for (int c = 2; c < ncols; c++) delta[1][c] = delta[0][c];
    while (!q.empty()) {
        int u = q.front();
        q.pop_front();
        for (int c = 2; c < ncols; c++) {
            int v = t.child[u][c];
            if (v >= 0) {
                fail[v] = delta[fail[u]][c];
                delta[u][c] = v;
                q.push_back(v);
            } else {
                delta[u][c] = delta[fail[u]][c];
            }
        }
    }

    // ---- outputs: the patterns that are suffixes of the node's reversed string,
    //      i.e. prefixes of the text from the current position
    std::vector<std::vector<int>> out_code(S, std::vector<int>(lk + 1, -1));
    for (int s = 2; s < S; s++) {
        const std::vector<uint8_t>& u = t.str[s];  // reversed text read so far (a suffix of it)
        for (int L = 1; L <= (int)u.size() && L <= lk; L++) {
            // pattern = reverse of the last L bytes of u
            std::string p;
            for (int k = (int)u.size() - 1; k >= (int)u.size() - L; k--) p.push_back((char)u[k]);
            auto it = seen.find(p);
            if (it != seen.end()) out_code[s][L] = it->second;
        }
    }
    out_code[1][1] = 0;  // one-byte-only state: a one-byte code starts here (code from CODE1)

    // ---- emit the image
    TableHeader h;
    memset(&h, 0, sizeof h);
    h.lmax = (uint32_t)lmax;
    h.lk = (uint32_t)lk;
    h.nstates = (uint32_t)S;
    h.ncols = (uint32_t)ncols;
    h.ncodes = (uint32_t)ncodes;
    uint32_t o = sizeof(TableHeader);
    h.off_len = o;   o = align16(o + 256);
    h.off_col = o;   o = align16(o + 256);
    h.off_code1 = o; o = align16(o + 256);
    h.off_trans = o; o = align16(o + (uint32_t)(S * ncols * 2));
    h.off_outk = o;  o = align16(o + (uint32_t)(S * lk));
    h.off_code = o;  o = align16(o + (uint32_t)(S * lk));
    h.off_exp = o;   o = align16(o + 256 * kExpStride);
    h.blob_bytes = o;
    std::vector<uint8_t>& blob = *blob_out;
    blob.assign(o, 0);
    memcpy(blob.data(), &h, sizeof h);
    for (int b = 0; b < 256; b++) {
        blob[h.off_len + b] = len[b];
        blob[h.off_col + b] = (uint8_t)col[b];
        blob[h.off_code1 + b] = code1[b];
        memcpy(&blob[h.off_exp + b * kExpStride], exp + b * kExpStride, (size_t)len[b]);
    }
    uint16_t* trans = (uint16_t*)&blob[h.off_trans];
    int8_t* outk = (int8_t*)&blob[h.off_outk];
    uint8_t* code = &blob[h.off_code];
    for (int s = 0; s < S; s++) {
        for (int c = 0; c < ncols; c++) trans[s * ncols + c] = (uint16_t)delta[s][c];
        for (int L = 1; L <= lk; L++) {
            int cd = out_code[s][L];
            outk[s * lk + (L - 1)] = cd >= 0 ? (int8_t)(31 - L) : (int8_t)-1;
            code[s * lk + (L - 1)] = cd > 0 ? (uint8_t)cd : 0;
        }
    }
    return ZS_OK;
}

// C-callable form for checks without a GPU: compile into a caller buffer.
// Returns ZS_OK and *size, ZS_ENOSPC if cap is too small, or ZS_EINVAL.
extern "C" int zsi_compile_dict_c(const uint8_t* len, const uint8_t* exp, uint8_t* out, uint64_t cap,
                                  uint64_t* size) {
    std::vector<uint8_t> blob;
    int rc = zsi_compile_dict(len, exp, &blob);
    if (rc != ZS_OK) return rc;
    *size = blob.size();
    if (blob.size() > cap) return ZS_ENOSPC;
    memcpy(out, blob.data(), blob.size());
    return ZS_OK;
}
