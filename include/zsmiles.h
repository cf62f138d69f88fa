/*
 * zsmiles.h - C ABI of the MI355X (gfx950) ZSMILES codec.
 *
 * The codec is the one of Accordi et al., "ZSMILES: an approach for efficient
 * SMILES storage for random access in Virtual Screening": one fixed,
 * input-independent dictionary maps printable code bytes to SMILES patterns;
 * every line (one SMILES) is compressed on its own, so line k of the output
 * is line k of the input and lines can be cut, combined and read at random
 * (Sec. I).  Compression optionally renumbers ring-closure IDs first
 * (Sec. IV-A), then takes a minimum-length parse of the line into codes and
 * escapes (Sec. IV-D-1); decompression is a table lookup per byte
 * (Sec. IV-D-2).
 *
 * Buffers.  A buffer holds lines, each ended by '\n'.  An index `off` of
 * n+1 uint64 entries frames n lines: line k is bytes [off[k], off[k+1]-1)
 * and byte off[k+1]-1 is its newline.  Offsets are absolute positions in the
 * buffer, so a sub-range of lines can be passed without copying.  The last
 * line may end at a virtual newline one past the buffer (off[n] =
 * in_bytes + 1); that byte is never read.  Output buffers use the same
 * framing and always start at out_off[0] = 0.
 *
 * Memory and streams.  Every pointer named in, out, in_off, out_off, ids,
 * ws, res or n_lines_out is DEVICE memory owned by the caller.  Every compute
 * call only enqueues work on `stream` (a hipStream_t passed as void*, NULL =
 * the default stream) and returns at once; it makes no allocation and no
 * synchronisation, so a sequence of calls can be captured into a HIP graph.
 * The return value reports problems visible on the host (bad arguments);
 * problems in the data are written to the device-resident zs_result `res`,
 * valid once the stream has reached the end of the call.
 *
 * Errors in the data.  A line that is badly framed (ZS_EINVAL), or holds a
 * byte outside 0x20..0x7E when compressing, or an undefined code, a dangling
 * escape or an escaped byte outside 0x20..0x7E when decompressing
 * (ZS_ECORRUPT), produces an empty output line; res->first_bad is the index
 * of the first such line (request index for zs_decompress_lines) and
 * res->code its code.  All other lines are still processed normally.  When no
 * line is bad and the output does not fit out_cap, res->code is ZS_ENOSPC,
 * out_off is still complete and out holds no useful bytes.
 *
 * Size-only mode: out == NULL computes out_off only (exact output sizes, used
 * for admission by footprint).
 *
 * Workspace: `ws` is caller-owned device scratch of at least
 * zs_workspace_bytes(op, n) bytes (n = lines, or ids for
 * zs_decompress_lines), 256-byte aligned (as hipMalloc returns it; a null
 * or misaligned ws is ZS_EINVAL); its contents need no initialisation.
 * Calls that share a workspace must not overlap in time.
 *
 * Thread safety: a zs_dict is immutable after creation and may be used by
 * many streams at once.
 */
#ifndef ZSMILES_H
#define ZSMILES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ZS_OK = 0,
    ZS_EINVAL = -1,   /* bad argument, bad framing, id out of range, bad dictionary */
    ZS_ENOSPC = -2,   /* output larger than out_cap (or index larger than off_cap) */
    ZS_ECORRUPT = -3, /* data that is not a SMILES line / not a compressed line    */
    ZS_EDEVICE = -4,  /* a HIP runtime call failed                                 */
    ZS_ENOMEM = -5    /* host or device allocation failed (dictionary creation)    */
} zs_status;

#define ZS_LMAX_CAP 16u      /* longest expansion a dictionary may hold              */
#define ZS_MAX_LINE 4096u    /* longest input line (bytes, newline excluded) accepted */
/* Longest compressed line (bytes, newline excluded): zs_compress never emits a
 * longer one (a line whose compressed form would be longer is bad, ZS_EINVAL:
 * only ring renumbering that lengthens a line gets past 2 * ZS_MAX_LINE, the
 * form of a longest line with every byte escaped), and the decoders take
 * every line up to it (a longer one is bad, ZS_EINVAL). */
#define ZS_MAX_CLINE 8192u
#define ZS_F_PREPROCESS 0x1u /* renumber ring IDs before compressing (Sec. IV-A)      */

/* Operations for zs_workspace_bytes. */
#define ZS_OP_COMPRESS 1
#define ZS_OP_DECOMPRESS 2
#define ZS_OP_DECOMPRESS_LINES 3
#define ZS_OP_INDEX 4

typedef struct zs_dict zs_dict;

/* Result word written by every compute call (device memory, 16 bytes). */
typedef struct {
    int32_t code;      /* zs_status of the data                          */
    int32_t reserved;
    int64_t first_bad; /* first bad line (or request) index, -1 if none  */
} zs_result;

/*
 * Create a dictionary (Sec. IV-B, IV-C: one fixed table shared by every
 * buffer).  len[b] is the expansion length of code byte b (0 = b is not a
 * code); exp[b*16 .. b*16+len[b]) its expansion.  Both are HOST arrays,
 * copied.  Rules (violations return ZS_EINVAL, *out untouched): code bytes
 * are printable, 0x21..0x7E or 0xA1..0xFF (0x20 is the escape, 0x0A the
 * separator); expansions are 1..16 bytes of 0x21..0x7E; no two codes share an
 * expansion; the matcher built from the patterns must fit the on-chip budget
 * (at most 4096 automaton states and 32 KiB of transition table).  The device
 * copy lives on the device current at the call.  Returns ZS_EDEVICE or
 * ZS_ENOMEM if the upload fails.
 */
zs_status zs_dict_create(const uint8_t *len, const uint8_t *exp, zs_dict **out);
void zs_dict_destroy(zs_dict *d);
/* Longest expansion of the dictionary (0 for an empty one). */
int zs_dict_lmax(const zs_dict *d);

/* Worst-case sizes, for sizing output buffers without a size-only pass. */
uint64_t zs_compress_bound(uint64_t in_bytes, uint64_t n_lines);
uint64_t zs_decompress_bound(const zs_dict *d, uint64_t in_bytes, uint64_t n_lines);
/* Workspace bytes for an operation over n lines (or n ids). */
size_t zs_workspace_bytes(int op, uint64_t n);

/*
 * Compress n_lines lines of `in` (in_bytes long, framed by in_off[0..n]).
 * flags: ZS_F_PREPROCESS renumbers ring-closure IDs first (Sec. IV-A).  Each
 * line is replaced by the shortest string of codes and escapes (' ' + byte)
 * that decodes to it, the parse that takes the longest code first among the
 * shortest ones (Sec. IV-D-1).  Output framing as described above;
 * out_off has n_lines+1 entries.  Lines longer than ZS_MAX_LINE, and lines
 * whose compressed form would be longer than ZS_MAX_CLINE, are bad
 * (ZS_EINVAL).
 */
zs_status zs_compress(const zs_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                      uint64_t n_lines, uint8_t *out, uint64_t out_cap, uint64_t *out_off, uint32_t flags,
                      void *ws, size_t ws_bytes, zs_result *res, void *stream);

/* Decompress every line (Sec. IV-D-2).  out_off has n_lines+1 entries.  A
 * compressed line longer than ZS_MAX_CLINE is bad (ZS_EINVAL). */
zs_status zs_decompress(const zs_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                        uint64_t n_lines, uint8_t *out, uint64_t out_cap, uint64_t *out_off, void *ws,
                        size_t ws_bytes, zs_result *res, void *stream);

/*
 * Random access (Sec. I: separable lines): decompress lines ids[0..n_ids) of
 * a compressed buffer and pack them in request order; out_off has n_ids+1
 * entries.  Ids may repeat and come in any order; an id >= n_lines is a bad
 * request (ZS_EINVAL, empty output line).
 */
zs_status zs_decompress_lines(const zs_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                              uint64_t n_lines, const uint64_t *ids, uint64_t n_ids, uint8_t *out,
                              uint64_t out_cap, uint64_t *out_off, void *ws, size_t ws_bytes, zs_result *res,
                              void *stream);

/*
 * zs_decompress_lines without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, output, result word
 * and errors as zs_decompress_lines, minus ws/ws_bytes: the call's scratch
 * (a header and one word per tile, about 545 KiB) is a static array that
 * the library holds on each device it runs on until the process ends.  It
 * allocates nothing and clears its scratch with a kernel.  n_ids above
 * ZS_NOALLOC_MAX_IDS returns ZS_EINVAL before anything is enqueued.  Every
 * call on one device shares that device's scratch: calls that overlap in
 * time on one device (different streams, or host threads) race and give
 * wrong results; serialise them, e.g. on one stream.
 */
#define ZS_NOALLOC_MAX_IDS (1u << 24)
zs_status zs_decompress_lines_noalloc(const zs_dict *d, const uint8_t *in, uint64_t in_bytes,
                                      const uint64_t *in_off, uint64_t n_lines, const uint64_t *ids,
                                      uint64_t n_ids, uint8_t *out, uint64_t out_cap, uint64_t *out_off,
                                      zs_result *res, void *stream);

/*
 * Build the line index of a newline-separated buffer (one SMILES per line,
 * Sec. I): off[0] = 0, off[k+1] = one past the k-th newline; a last line
 * without newline ends at the virtual newline len+1.  *n_lines_out (device
 * uint64) receives the number of lines.  At most off_cap entries are written;
 * if lines+1 > off_cap, res->code is ZS_ENOSPC.  ws: zs_workspace_bytes(
 * ZS_OP_INDEX, len).
 */
zs_status zs_index_lines(const uint8_t *buf, uint64_t len, uint64_t *off, uint64_t off_cap,
                         uint64_t *n_lines_out, void *ws, size_t ws_bytes, zs_result *res, void *stream);

/*
 * Length-binned compression, for batches whose line lengths are very uneven
 * (the paper's compressor takes one block per SMILES, Sec. IV-E; here lines are
 * grouped by length so that the lanes of a wavefront hold lines of similar
 * length).  On the device, the lines are sorted by raw length into cfg->nbins
 * bins (a stable counting sort), every bin is compressed with its own tile
 * shape, longest bin first, into a staging area of the workspace, and a last
 * pass writes the lines back in input order.  The output (out, out_off, res)
 * is identical to zs_compress's for every input; size-only mode and ENOSPC
 * behave the same.  ws: at least zs_binned_workspace_bytes(n_lines, out_cap)
 * bytes, 256-byte aligned (it holds the staging copy of the output).
 */
#define ZS_MAX_BINS 8
typedef struct {
    uint32_t nbins;                        /* 1..ZS_MAX_BINS                                      */
    uint32_t edges[ZS_MAX_BINS - 1];       /* ascending raw-length bounds: bin i holds lengths in */
                                           /* [edges[i-1], edges[i]) (edges[-1] = 0, last open)   */
    uint32_t lines_per_tile[ZS_MAX_BINS];  /* per bin, 32..256: lines (lanes) per workgroup tile  */
    uint32_t large_lds[ZS_MAX_BINS];       /* per bin, where a tile's lines are held: 0 LDS (3    */
                                           /* workgroups per CU), 1 a larger LDS batch (2 per     */
                                           /* CU), 2 global memory (the workspace: up to 256 KiB  */
                                           /* of lines per tile, so a tile of long lines keeps    */
                                           /* every lane busy; LDS then holds the automaton)      */
} zs_bin_config;

size_t zs_binned_workspace_bytes(uint64_t n_lines, uint64_t out_cap);
zs_status zs_compress_binned(const zs_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                             uint64_t n_lines, uint8_t *out, uint64_t out_cap, uint64_t *out_off, uint32_t flags,
                             const zs_bin_config *cfg, void *ws, size_t ws_bytes, zs_result *res, void *stream);

/*
 * Autotuner for zs_compress_binned: times a set of configurations (bin edges
 * from the quantiles of the line lengths, lines per tile, LDS layout) on the
 * given lines, which should be a sample of the workload, and returns the
 * fastest in *best (and its time, ms, in *best_ms; the plain zs_compress time
 * on the same lines in *plain_ms).  Unlike the compute calls it allocates
 * device memory for its trials and synchronises; it runs on `stream`.
 * n_tried receives the number of configurations timed.
 */
zs_status zs_autotune_binned(const zs_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                             uint64_t n_lines, uint32_t flags, zs_bin_config *best, double *best_ms,
                             double *plain_ms, uint32_t *n_tried, void *stream);

/*
 * HIP graphs of codec calls.  zs_graph_begin starts capturing the work that
 * the following calls enqueue on `stream` (not the NULL stream);
 * zs_graph_end stops and instantiates it.  zs_graph_launch replays the whole
 * sequence with one launch; the captured calls read and write the same
 * buffers on every replay.  Every kernel of the library may be captured (the
 * library clears its counters with kernels, not memset nodes).
 */
typedef struct zs_graph zs_graph;
zs_status zs_graph_begin(void *stream);
zs_status zs_graph_end(void *stream, zs_graph **out);
zs_status zs_graph_launch(zs_graph *g, void *stream);
void zs_graph_destroy(zs_graph *g);

/*
 * Request loop (one GPU).  Compressed shards stay resident in device memory
 * (registered with zs_server_add_shard, owned by the caller) and share one
 * dictionary; random-access decompression requests (ids of a shard) and
 * compression requests (new lines) may be submitted from any host thread.  A
 * scheduler thread admits them in arrival order into `slots` HIP streams, so
 * the work of many requests overlaps on the device.  Admission is by device
 * footprint: a request first runs its call in size-only mode, then takes an
 * output buffer of the exact size from a device arena of `device_bytes`
 * (made at creation: the loop itself allocates nothing).  Inputs are copied
 * at submission into a pinned host arena of `host_bytes`; results come back
 * there.  zs_server_wait blocks until a request is done and describes its
 * result, which stays valid until zs_server_release.  Every result equals
 * what the same call gives on its own.  A request whose inputs fit but
 * whose output (known after sizing) can never be held by the arenas, even
 * with nothing else in them, ends with code ZS_ENOSPC and no offsets or
 * bytes (off and data NULL).
 */
typedef struct zs_server zs_server;
typedef struct {
    uint32_t slots;         /* concurrent requests (streams), 1..64 */
    uint64_t device_bytes;  /* device arena for request buffers     */
    uint64_t host_bytes;    /* pinned host arena for inputs/outputs */
} zs_server_config;
typedef struct {
    int32_t code;           /* zs_status of the data (as zs_result)        */
    int64_t first_bad;
    uint64_t n;             /* ids or lines                                 */
    const uint64_t *off;    /* host: n+1 output offsets                     */
    const uint8_t *data;    /* host: output bytes                           */
    uint64_t bytes;
    double t_submit, t_admit, t_done;  /* seconds, one steady clock         */
    uint64_t footprint;     /* device bytes the request held                */
} zs_reply;
typedef struct {
    uint64_t submitted, admitted, completed, deferred;
    uint64_t peak_device_bytes, device_bytes_in_use;
    double busy_s;          /* sum over requests of admit-to-done time      */
} zs_server_stats;

zs_status zs_server_create(const zs_dict *d, const zs_server_config *cfg, zs_server **out);
zs_status zs_server_add_shard(zs_server *s, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                              uint64_t n_lines, uint32_t *shard);
/* ids: host array, copied; ZS_ENOSPC if the request can never fit the arenas. */
zs_status zs_server_submit_decompress(zs_server *s, uint32_t shard, const uint64_t *ids, uint64_t n_ids,
                                      uint64_t *ticket);
/* lines, off: host arrays (off[0..n], absolute in lines), copied. */
zs_status zs_server_submit_compress(zs_server *s, const uint8_t *lines, uint64_t bytes, const uint64_t *off,
                                    uint64_t n_lines, uint32_t flags, uint64_t *ticket);
zs_status zs_server_wait(zs_server *s, uint64_t ticket, zs_reply *out);
void zs_server_release(zs_server *s, uint64_t ticket);
zs_status zs_server_get_stats(zs_server *s, zs_server_stats *out);
/* Finishes the admitted and queued requests, then frees everything. */
void zs_server_destroy(zs_server *s);

/*
 * Ring-ID pre-processing alone (Sec. IV-A): every line of `in` is written
 * with its ring-closure labels renumbered, exactly the form zs_compress
 * parses under ZS_F_PREPROCESS (and the form decompression gives back).
 * Framing, errors (bad lines come out empty), size-only mode and ENOSPC as
 * for zs_compress; a line grows at most 3x (a digit label may become %nn),
 * so 3 * in_bytes + n_lines bytes always suffice.  ws: zs_workspace_bytes(
 * ZS_OP_COMPRESS, n_lines).
 */
zs_status zs_preprocess(const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off, uint64_t n_lines,
                        uint8_t *out, uint64_t out_cap, uint64_t *out_off, void *ws, size_t ws_bytes,
                        zs_result *res, void *stream);

/*
 * Post-processing of decompressed lines.  The paper's execution flow
 * (Sec. IV-D) lets decompressed SMILES be "optionally post-processed" without
 * defining the step; the definition taken here: ring-closure labels are
 * renumbered the way SMILES writers usually number them - reading left to
 * right, a ring's opening label takes the smallest label >= 1 not held by a
 * ring open at that point, and its closing label repeats it (1..9 as a digit,
 * 10..99 as %nn).  Tokens, pairing and malformed lines (left unchanged) as in
 * pre-processing; a line that would need label 100 is left unchanged.  Lines
 * longer than ZS_MAX_LINE are bad (ZS_EINVAL).  Arguments, framing, errors,
 * size-only mode and workspace as for zs_preprocess (3 * in_bytes + n_lines
 * bytes always suffice).
 */
zs_status zs_postprocess(const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off, uint64_t n_lines,
                         uint8_t *out, uint64_t out_cap, uint64_t *out_off, void *ws, size_t ws_bytes,
                         zs_result *res, void *stream);

/*
 * Dictionary generation, Algorithm 1 of Sec. IV-C, on the device.  Counts
 * every substring of lmin..lmax bytes of every line (overlapping occurrences
 * included; of the pre-processed lines when flags has ZS_F_PREPROCESS, as the
 * paper trains its dictionaries, Sec. V-B), then T times takes the substring
 * of highest rank occ * (len - overlap) (Eq. (1)), where overlap is the
 * longest common substring with any pattern taken before (the reading of the
 * paper's update_rank); ties go to the longer, then the bytewise smaller
 * substring.  It stops early when no substring has a positive rank.
 * Outputs (device): pat[t*16 .. t*16+pat_len[t]) is the t-th pattern taken,
 * zero padded to 16 bytes; *n_chosen (uint32) how many were taken.  The
 * caller assigns code bytes (Sec. IV-B: e.g. after the SMILES alphabet).
 * Lines follow the rules of zs_compress (bytes 0x20..0x7E, at most
 * ZS_MAX_LINE); any bad line makes the call fail: res->code and first_bad
 * as for compression, *n_chosen = 0.  1 <= lmin <= lmax <= 16, T <=
 * ZS_TRAIN_MAX_T, else ZS_EINVAL.  ws: zs_train_workspace_bytes(...) bytes,
 * which grows with in_bytes * (lmax - lmin + 1) (an open-addressing table with
 * room for every occurrence: about 40 bytes per occurrence, 3x that with
 * pre-processing, whose lines may grow).  Enqueue-only like the other calls
 * (2T + 6 kernel launches).
 */
#define ZS_TRAIN_MAX_T 4096u
size_t zs_train_workspace_bytes(uint64_t in_bytes, uint64_t n_lines, uint32_t lmin, uint32_t lmax, uint32_t flags);
zs_status zs_train_patterns(const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off, uint64_t n_lines,
                            uint32_t flags, uint32_t lmin, uint32_t lmax, uint32_t T, uint8_t *pat,
                            uint8_t *pat_len, uint32_t *n_chosen, void *ws, size_t ws_bytes, zs_result *res,
                            void *stream);

/* Human-readable name of a status code. */
const char *zs_status_str(int code);

#ifdef __cplusplus
}
#endif
#endif /* ZSMILES_H */
