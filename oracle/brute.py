"""oracle/brute.py - TEST INFRASTRUCTURE ONLY.

Independent, deliberately naive checks used to pin the C oracle.  Nothing here
calls zs_oracle.c, and the algorithms are different ones:

* brute_compress enumerates every parse of a short string into dictionary
  codes and escapes (Sec. IV-D-1), keeps those of minimum output length and
  returns the one whose sequence of consumed lengths is lexicographically
  greatest (reading "T1");
* dijkstra_cost builds the graph G of Sec. IV-D-1 explicitly and runs
  Dijkstra with a binary heap;
* preprocess_alt assigns ring IDs by a streaming rule: keep, for every ID, the
  position of the latest closing label that received it; a closing ring takes
  the smallest ID whose latest close is before the ring's opening label.  This
  equals the oracle's "smallest ID not held by a ring closed inside me", by a
  one-line argument (an ID is held by a ring closed inside R iff its latest
  close before R's closing label falls after R's opening label);
* postprocess_alt computes the post-processing labels from ring intervals
  instead of a left-to-right walk: a ring's label is the smallest label >= 1
  not used by a ring whose interval contains the ring's opening label, taking
  the rings in order of their opening labels;
* ring_intervals / omega give the ring structure of a line for properties
  such as "nested rings get distinct IDs, inner lower" (Sec. II, Sec. IV-A).
"""
import heapq


def _codes_by_exp(entries):
    return {bytes(e): c for c, e in entries.items()}


def all_parses(entries, s):
    """Yield (output bytes, tuple of consumed lengths) for every parse of s."""
    inv = _codes_by_exp(entries)
    lens = sorted({len(e) for e in inv})
    s = bytes(s)

    def rec(i):
        if i == len(s):
            yield b"", ()
            return
        # escape: a space, then the byte itself
        for out, ls in rec(i + 1):
            yield b" " + s[i:i + 1] + out, (1,) + ls
        for L in lens:
            if i + L <= len(s) and s[i:i + L] in inv:
                code = bytes([inv[s[i:i + L]]])
                for out, ls in rec(i + L):
                    yield code + out, (L,) + ls

    yield from rec(0)


def brute_compress(entries, s):
    best = None
    for out, ls in all_parses(entries, s):
        key = (len(out), tuple(-x for x in ls))
        if best is None or key < best[0]:
            best = (key, out)
    return best[1]


def brute_min_len(entries, s):
    return min(len(out) for out, _ in all_parses(entries, s))


def dijkstra_cost(entries, s):
    """Shortest path from node 0 to node len(s) in G (Sec. IV-D-1)."""
    inv = _codes_by_exp(entries)
    s = bytes(s)
    m = len(s)
    adj = [[] for _ in range(m + 1)]
    for i in range(m):
        adj[i].append((i + 1, 2))
        for j in range(i + 1, m + 1):
            if s[i:j] in inv:
                adj[i].append((j, 1))
    dist = [None] * (m + 1)
    heap = [(0, 0)]
    while heap:
        d, u = heapq.heappop(heap)
        if dist[u] is not None:
            continue
        dist[u] = d
        for v, w in adj[u]:
            if dist[v] is None:
                heapq.heappush(heap, (d + w, v))
    return dist[m]


def _label_tokens(s):
    """Ring-closure label tokens (start, end, value) outside brackets, or None if malformed."""
    toks = []
    depth = 0
    i = 0
    s = bytes(s)
    while i < len(s):
        ch = s[i]
        if ch == ord("["):
            depth += 1
            if depth > 1:
                return None
        elif ch == ord("]"):
            depth -= 1
            if depth < 0:
                return None
        elif depth == 0 and 48 <= ch <= 57:
            toks.append((i, i + 1, ch - 48))
        elif depth == 0 and ch == ord("%"):
            if i + 2 < len(s) and 48 <= s[i + 1] <= 57 and 48 <= s[i + 2] <= 57:
                toks.append((i, i + 3, (s[i + 1] - 48) * 10 + (s[i + 2] - 48)))
                i += 2
            else:
                return None
        i += 1
    if depth != 0:
        return None
    return toks


def ring_intervals(s):
    """List of (open token index, close token index) in closing order, or None."""
    toks = _label_tokens(s)
    if toks is None:
        return None
    pending = {}
    rings = []
    for ti, (_, _, v) in enumerate(toks):
        if v in pending:
            rings.append((pending.pop(v), ti))
        else:
            pending[v] = ti
    if pending:
        return None
    return rings


def omega(s):
    """Largest number of rings open at once (a ring is open from its opening to its closing label)."""
    rings = ring_intervals(s)
    if not rings:
        return 0
    events = []
    for o, c in rings:
        events.append((o, 1))
        events.append((c, -1))
    events.sort()
    cur = best = 0
    for _, e in events:
        cur += e
        best = max(best, cur)
    return best


def preprocess_alt(s):
    """Ring-ID reuse (Sec. IV-A) by the streaming 'latest close per ID' rule."""
    s = bytes(s)
    toks = _label_tokens(s)
    if toks is None:
        return s
    open_at = {}
    latest_close = {}
    new_id = {}
    for ti, (_, _, v) in enumerate(toks):
        if v not in open_at:
            open_at[v] = ti
            continue
        oi = open_at.pop(v)
        rid = 0
        while latest_close.get(rid, -1) > oi:
            rid += 1
        if rid >= 100:
            return s
        latest_close[rid] = ti
        new_id[oi] = rid
        new_id[ti] = rid
    if open_at:
        return s
    out = bytearray()
    pos = 0
    for ti, (a, b, _) in enumerate(toks):
        out += s[pos:a]
        rid = new_id[ti]
        out += (b"%d" % rid) if rid < 10 else (b"%%%02d" % rid)
        pos = b
    out += s[pos:]
    return bytes(out)


def decompress_ref(entries, c):
    """Sec. IV-D-2 written out once more for tiny cases; None if corrupt."""
    c = bytes(c)
    out = bytearray()
    j = 0
    while j < len(c):
        if c[j] == 32:
            if j + 1 >= len(c) or not (32 <= c[j + 1] <= 126):
                return None
            out.append(c[j + 1])
            j += 2
        else:
            if c[j] not in entries:
                return None
            out += entries[c[j]]
            j += 1
    return bytes(out)


def postprocess_alt(s):
    """Writers' ring numbering (our definition of post-processing) from ring intervals."""
    s = bytes(s)
    toks = _label_tokens(s)
    rings = ring_intervals(s)
    if toks is None or rings is None:
        return s
    label = {}
    for o, c in sorted(rings):  # by opening token
        used = {label[(o2, c2)] for (o2, c2) in label if o2 < o < c2}
        v = 1
        while v in used:
            v += 1
        if v > 99:
            return s
        label[(o, c)] = v
    new_of_tok = {}
    for (o, c), v in label.items():
        new_of_tok[o] = v
        new_of_tok[c] = v
    out = bytearray()
    i = 0
    ti = 0
    while i < len(s):
        if ti < len(toks) and toks[ti][0] == i:
            v = new_of_tok[ti]
            out += (b"%d" % v) if v < 10 else (b"%%%02d" % v)
            i = toks[ti][1]
            ti += 1
        else:
            out.append(s[i])
            i += 1
    return bytes(out)
