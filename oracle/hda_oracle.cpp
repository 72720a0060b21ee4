// Allocator replay oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, sequential CPU model of the allocators in "Host-Based
// Allocators for Device Memory" (Bell, Kumar, Gill): first fit, next fit and
// best fit over an address-ordered free list (Sec. II-A, Sec. IV, Alg. 1-3),
// segregated fit over address-keyed block records threaded into per-class
// free lists with a class-availability bitmap (Sec. III-C, Sec. V-A,
// Alg. 4-5), and two-level segregated fit (TLSF, Sec. V-B), the same
// machinery with each power-of-two class split linearly and a two-level
// bitmap lookup, and the bitmask allocator with a next-fit search (Sec.
// III-B): one flag per granule, an allocation takes the first run of free
// granules of the request's length found scanning from where the last one
// ended.  No metadata lives in the managed memory: the arena is never
// touched, only described.
//
// Only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark may load this library.  The GPU path shares no code with it.
//
// Plain library containers are used on purpose (std::map keyed by address
// plays the role of the paper's sorted lists and of its address-keyed hash
// table); nothing is blocked, fused or reordered.
//
// Readings where the paper is silent or inconsistent (each applied here):
//  * Sizes are normalised to s = max(g, roundup(req, g)); a request larger
//    than the arena fails (the paper passes sizes through unchanged).
//  * The block handed out is the low end of the chosen free block (Alg. 1,
//    Alg. 4: the free entry's address advances by the size).
//  * Best fit picks the smallest block with size >= s, lowest address among
//    equals; an exact size match is taken (Sec. II-A prose; Alg. 3's loop
//    exits on an exact match and starts from a sentinel).
//  * Next fit keeps a rover byte address, set to a+s after every successful
//    allocation and left alone otherwise; a search starts at the first free
//    block whose end lies above the rover and wraps around once.
//  * Deallocation merges with the free predecessor when it ends exactly at
//    the freed address and with the free successor when it starts exactly at
//    the freed end; in the three-way case the successor entry is removed
//    (Alg. 2 with equality tests).
//  * Segregated fit: class k holds sizes in [2^k, 2^(k+1)) bytes; a request
//    of s bytes is served from the lowest non-empty class >= ceil(log2 s)
//    found with find-first-set on the bitmap, never from class
//    ceil(log2 s)-1 (Sec. II-B; the "nearly 4x larger" remark of Sec. V-A
//    fixes this 0-based class index).  Lists are LIFO: pop and push at the
//    head (Alg. 4, Alg. 5).  A class bit is cleared exactly when its list
//    becomes empty.  On free, free neighbours are unlinked from their lists
//    first and the merged block is always pushed at the head of the list of
//    floor(log2 size).  The null link is -1 (offset 0 is a valid address).
//  * TLSF (Sec. V-B; the paper gives no second-level count): every power of
//    two is split into 32 linear sub-classes (second-level index 5, the
//    default of the TLSF authors' implementation).  A block of b bytes is in
//    class (fl, sl) with fl = floor(log2 b) and sl = (b >> (fl-5)) - 32
//    (b << (5-fl) when fl < 5, so that each such class holds one size).  A
//    request of s bytes is first rounded up to the next sub-class boundary,
//    s + 2^(fl-5) - 1 for fl >= 5 (nothing below), and its class (fl, sl)
//    taken from that; every block of that class or a higher one is then at
//    least s.  The lookup consults the second-level bitmap of fl for a
//    sub-class >= sl, and otherwise the first-level bitmap for the lowest
//    fl' > fl and that level's lowest sub-class.  Lists, splitting, merging
//    and pushing are those of segregated fit; a first-level bit is set
//    exactly when one of its sub-class lists is non-empty.
//  * Bitmask allocator (Sec. III-B; the search is next fit, as the paper
//    suggests): a rover (byte address), 0 at start, set to p + s after allocating
//    [p, p + s).  An allocation of s granules takes the lowest p >= rover
//    such that granules [p, p + s) are all free, else the lowest p >= 0
//    such that they are (wrapping once); on failure the rover stays.  Unlike
//    the list-based next fit it may cut the run from the middle of a free
//    block (the scan starts at the rover, not at the block's start).  Free
//    sets the granules' flags back, so merging is implicit.  The free flags
//    are kept here as the address-ordered list of maximal free runs, which
//    is exactly what the flags describe and what the state dump lists.
//  * No allocation ever fails with an error: a request nothing can satisfy
//    returns -1 and leaves the state (and the rover) unchanged.
//  * Partial deallocation (Sec. II-A, Alg. 2) is defined for the sequential
//    fits only: freeing x inside the live block [b, b+s), b < x, shrinks it
//    to [b, x) and releases [x, b+s) with the same merging as a whole block;
//    the block keeps its place in live[].  x must be a multiple of g.
//    Segregated fit and TLSF free exactly one keyed block (Alg. 5), so an
//    interior address is a bad free there.
//  * Replay driver (not part of the paper): a free request q < 0 carries
//    u = ~q, a uniform 32-bit draw r = u mod 2^32 and a cut c = u >> 32
//    (0 <= c < 2^31).  The victim is live[(r * L) >> 32] where live[] lists
//    the live blocks (append on success, swap-with-last removal on a whole
//    free) and L = |live|.  For the sequential fits the victim's first
//    t = floor(c * (s / g) / 2^31) granules stay live and the rest is freed
//    (t = 0: the whole block); segregated fit and TLSF ignore c.  The result is the
//    byte address freed.  With no live block the request does nothing and
//    yields -1.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

namespace {

constexpr int FF = 0, NF = 1, BF = 2, SF = 3, TLSF = 4, BITMAP = 5;
constexpr int SLI = 5, NSL = 1 << SLI;   // TLSF second level: 32 sub-classes
constexpr int64_t NIL = -1;
constexpr int E_INVAL = -2, E_BADFREE = -3;

int floor_log2(uint64_t x) {  // x >= 1
    int k = -1;
    while (x) { x >>= 1; ++k; }
    return k;
}
int ceil_log2(uint64_t x) {   // x >= 1: smallest k with 2^k >= x
    int k = 0;
    while ((uint64_t(1) << k) < x) ++k;
    return k;
}

struct SfRecord {             // Sec. III-C: what a block header would hold
    int64_t size;
    bool free;
    int64_t prev_adj;         // address of the block ending at this one's start
    int64_t next_free;        // free-list links (addresses)
    int64_t prev_free;
};

struct Heap {
    int algo;
    int64_t A, g;
    // in-use blocks, address -> size (the "used list")
    std::map<int64_t, int64_t> used;
    // replay-driver order of the live blocks
    std::vector<int64_t> live;
    // sequential fits: address-ordered free list, address -> size
    std::map<int64_t, int64_t> fl;
    int64_t rover = 0;
    // segregated fit / TLSF: address-keyed records, list heads, availability
    // bitmap (TLSF: first level, plus one second-level bitmap per level)
    std::map<int64_t, SfRecord> ht;
    std::vector<int64_t> head;
    uint64_t bitmap = 0;
    uint32_t sl_bitmap[64] = {};
    // instrumentation
    uint64_t examined = 0;    // free entries inspected by a fit search
    uint64_t touched = 0;     // segregated-fit records read or written

    Heap(int a, int64_t arena, int64_t align)
        : algo(a), A(arena), g(align), head(a == TLSF ? 64 * NSL : 64, NIL) {
        // Alg. 6: the free list starts as the single block [0, A).
        if (segregated()) {
            ht[0] = SfRecord{A, true, NIL, NIL, NIL};
            push(0);
        } else {
            fl[0] = A;
        }
    }

    bool segregated() const { return algo == SF || algo == TLSF; }

    // ---- size classes ----
    // TLSF class (fl, sl) of b >= 1 bytes, as the index fl * 32 + sl.
    static int tlsf_class(uint64_t b) {
        int fl = floor_log2(b);
        uint64_t sl = fl >= SLI ? (b >> (fl - SLI)) - NSL : (b << (SLI - fl)) - NSL;
        return fl * NSL + int(sl);
    }
    // The list a free block of `size` bytes belongs to.
    int cls(int64_t size) const {
        return algo == TLSF ? tlsf_class(uint64_t(size)) : floor_log2(uint64_t(size));
    }
    void mark(int c) {
        if (algo == TLSF) {
            sl_bitmap[c / NSL] |= uint32_t(1) << (c % NSL);
            bitmap |= uint64_t(1) << (c / NSL);
        } else {
            bitmap |= uint64_t(1) << c;
        }
    }
    void unmark(int c) {
        if (algo == TLSF) {
            sl_bitmap[c / NSL] &= ~(uint32_t(1) << (c % NSL));
            if (sl_bitmap[c / NSL] == 0) bitmap &= ~(uint64_t(1) << (c / NSL));
        } else {
            bitmap &= ~(uint64_t(1) << c);
        }
    }

    // ---- segregated-fit list primitives (Alg. 4, Alg. 5) ----
    void push(int64_t a) {
        SfRecord& r = ht.at(a);
        int c = cls(r.size);
        r.prev_free = NIL;
        r.next_free = head[c];
        if (head[c] != NIL) { ht.at(head[c]).prev_free = a; ++touched; }
        head[c] = a;
        mark(c);
        ++touched;
    }
    void unlink(int64_t a) {
        SfRecord& r = ht.at(a);
        int c = cls(r.size);
        if (r.prev_free != NIL) { ht.at(r.prev_free).next_free = r.next_free; ++touched; }
        else head[c] = r.next_free;
        if (r.next_free != NIL) { ht.at(r.next_free).prev_free = r.prev_free; ++touched; }
        if (head[c] == NIL) unmark(c);
        r.next_free = r.prev_free = NIL;
        ++touched;
    }

    // The list an allocation of s bytes pops from, or -1 (Alg. 4's bitmap
    // lookup; TLSF: the two-level lookup of Sec. V-B).
    int find_list(int64_t s) const {
        if (algo == SF) {
            int k = ceil_log2(uint64_t(s));
            uint64_t m = (k >= 64) ? 0 : (bitmap & (~uint64_t(0) << k));
            return m == 0 ? -1 : __builtin_ctzll(m);
        }
        int f0 = floor_log2(uint64_t(s));
        uint64_t r = uint64_t(s) + (f0 >= SLI ? (uint64_t(1) << (f0 - SLI)) - 1 : 0);
        int c = tlsf_class(r), fl = c / NSL, sl = c % NSL;
        if (fl >= 64) return -1;
        uint32_t slm = sl_bitmap[fl] & (~uint32_t(0) << sl);
        if (slm == 0) {
            uint64_t flm = fl + 1 >= 64 ? 0 : (bitmap & (~uint64_t(0) << (fl + 1)));
            if (flm == 0) return -1;
            fl = __builtin_ctzll(flm);
            slm = sl_bitmap[fl];
        }
        return fl * NSL + __builtin_ctz(slm);
    }

    // ---- allocation ----
    int64_t alloc(int64_t req) {
        if (req < 0 || req > A) return -1;
        int64_t s = (req + g - 1) / g * g;
        if (s == 0) s = g;
        if (s > A) return -1;
        int64_t a = segregated() ? alloc_sf(s) : algo == BITMAP ? alloc_bitmap(s) : alloc_seq(s);
        if (a >= 0) { used[a] = s; live.push_back(a); }
        return a;
    }

    int64_t alloc_seq(int64_t s) {
        auto pick = fl.end();
        if (algo == FF) {            // lowest address with size >= s
            for (auto it = fl.begin(); it != fl.end(); ++it) {
                ++examined;
                if (it->second >= s) { pick = it; break; }
            }
        } else if (algo == BF) {     // min (size, address) with size >= s
            for (auto it = fl.begin(); it != fl.end(); ++it) {
                ++examined;
                if (it->second >= s &&
                    (pick == fl.end() || it->second < pick->second)) pick = it;
                if (it->second == s) break;
            }
        } else {                     // NF: resume at the block holding the rover
            auto start = fl.begin();
            while (start != fl.end() && start->first + start->second <= rover) ++start;
            if (start == fl.end()) start = fl.begin();
            auto it = start;
            for (size_t n = 0; n < fl.size(); ++n) {
                ++examined;
                if (it->second >= s) { pick = it; break; }
                if (++it == fl.end()) it = fl.begin();
            }
        }
        if (pick == fl.end()) return -1;
        // Alg. 1: take the low end; shrink the free entry or remove it.
        int64_t a = pick->first, bsize = pick->second;
        fl.erase(pick);
        if (bsize > s) fl[a + s] = bsize - s;
        if (algo == NF) rover = a + s;
        return a;
    }

    // Sec. III-B: a run of s free granules, scanning from the rover, then
    // from the start.
    int64_t alloc_bitmap(int64_t s) {
        auto pick = fl.end();
        int64_t p = -1;
        for (auto it = fl.begin(); it != fl.end() && pick == fl.end(); ++it) {
            ++examined;
            int64_t from = std::max(it->first, rover);
            if (from + s <= it->first + it->second) { pick = it; p = from; }
        }
        for (auto it = fl.begin(); it != fl.end() && pick == fl.end(); ++it) {
            ++examined;
            if (it->second >= s) { pick = it; p = it->first; }
        }
        if (pick == fl.end()) return -1;
        int64_t a = pick->first, end = a + pick->second;
        fl.erase(pick);
        if (p > a) fl[a] = p - a;
        if (p + s < end) fl[p + s] = end - (p + s);
        rover = p + s;
        return p;
    }

    int64_t alloc_sf(int64_t s) {
        int c = find_list(s);
        if (c < 0) return -1;
        int64_t a = head[c];
        unlink(a);
        SfRecord& it = ht.at(a);
        it.free = false;
        ++touched;
        if (it.size > s) {           // split off the surplus, push it
            int64_t b = a + s, r = it.size - s, old_end = a + it.size;
            it.size = s;
            ht[b] = SfRecord{r, true, a, NIL, NIL};
            push(b);
            if (old_end < A) { ht.at(old_end).prev_adj = b; ++touched; }
        }
        return a;
    }

    // ---- deallocation ----
    int dealloc(int64_t x) {
        auto u = used.find(x);
        if (u == used.end()) return E_BADFREE;
        int64_t s = u->second;
        used.erase(u);
        auto lv = std::find(live.begin(), live.end(), x);
        *lv = live.back();
        live.pop_back();
        if (segregated()) dealloc_sf(x); else dealloc_seq(x, s);
        return 0;
    }

    // Alg. 2 for an address that may lie inside a live block: the block
    // holding x shrinks to end at x and the tail is released (sequential
    // fits); x at a block's start frees the whole block.
    int dealloc_partial(int64_t x) {
        auto u = used.upper_bound(x);
        if (u == used.begin()) return E_BADFREE;
        --u;
        int64_t b = u->first, s = u->second;
        if (x >= b + s) return E_BADFREE;
        if (x == b) return dealloc(x);
        if (segregated() || x % g != 0) return E_BADFREE;
        u->second = x - b;           // it.size = addr - it.addr
        dealloc_seq(x, b + s - x);   // size -= it.size
        return 0;
    }

    void dealloc_seq(int64_t x, int64_t s) {
        // Alg. 2: predecessor = last free block below x, successor = next.
        auto succ = fl.upper_bound(x);
        auto pred = (succ == fl.begin()) ? fl.end() : std::prev(succ);
        bool left = pred != fl.end() && pred->first + pred->second == x;
        bool right = succ != fl.end() && succ->first == x + s;
        if (left && right) {
            pred->second += s + succ->second;
            fl.erase(succ);
        } else if (left) {
            pred->second += s;
        } else if (right) {
            int64_t sz = succ->second;
            fl.erase(succ);
            fl[x] = s + sz;
        } else {
            fl[x] = s;
        }
    }

    void dealloc_sf(int64_t x) {
        SfRecord it = ht.at(x);
        ++touched;
        int64_t start = x, end = x + it.size, prev_adj = it.prev_adj;
        bool left = it.prev_adj != NIL && ht.at(it.prev_adj).free;
        bool right = end < A && ht.at(end).free;
        touched += (it.prev_adj != NIL) + (end < A);
        if (left) {
            int64_t l = it.prev_adj;
            unlink(l);
            start = l;
            prev_adj = ht.at(l).prev_adj;
            ht.erase(x);
        }
        if (right) {
            int64_t r = end;
            end = r + ht.at(r).size;
            unlink(r);
            ht.erase(r);
        }
        SfRecord& m = ht[start];
        m.size = end - start;
        m.free = true;
        m.prev_adj = prev_adj;
        if (end < A) { ht.at(end).prev_adj = start; ++touched; }
        push(start);
    }

    // ---- canonical state ----
    // [n_free, (addr,size)*n_free by address, n_live, (addr,size)*n_live in
    //  live order, rover (next fit) or -1, bitmap (segregated fit; TLSF: the
    //  first level) or 0, segregated fit / TLSF only: for each list (64 or
    //  64 * 32 of them, class index order): len, addresses head->tail]
    std::vector<int64_t> dump() const {
        std::vector<int64_t> o;
        std::vector<std::pair<int64_t, int64_t>> fb;
        if (segregated()) {
            for (auto& kv : ht) if (kv.second.free) fb.push_back({kv.first, kv.second.size});
        } else {
            for (auto& kv : fl) fb.push_back(kv);
        }
        o.push_back(int64_t(fb.size()));
        for (auto& p : fb) { o.push_back(p.first); o.push_back(p.second); }
        o.push_back(int64_t(live.size()));
        for (int64_t a : live) { o.push_back(a); o.push_back(used.at(a)); }
        o.push_back(algo == NF || algo == BITMAP ? rover : -1);
        o.push_back(segregated() ? int64_t(bitmap) : 0);
        if (segregated()) {
            for (int c = 0; c < int(head.size()); ++c) {
                std::vector<int64_t> lst;
                for (int64_t a = head[c]; a != NIL; a = ht.at(a).next_free) lst.push_back(a);
                o.push_back(int64_t(lst.size()));
                o.insert(o.end(), lst.begin(), lst.end());
            }
        }
        return o;
    }
};

bool valid_params(int algo, int64_t arena, int64_t align) {
    if (algo < 0 || algo > 5) return false;
    if (align <= 0 || (align & (align - 1))) return false;
    if (arena <= 0 || arena % align) return false;
    if (arena / align >= (int64_t(1) << 32)) return false;
    return true;
}

// Replay one heap's requests in order (see the replay-driver reading above).
void replay_one(Heap& h, int64_t n, const int64_t* req, int64_t* res) {
    for (int64_t i = 0; i < n; ++i) {
        int64_t q = req[i];
        if (q >= 0) {
            res[i] = h.alloc(q);
        } else if (h.live.empty()) {
            res[i] = -1;
        } else {
            uint64_t u = ~uint64_t(q);
            uint64_t r = uint32_t(u), c = u >> 32;
            uint64_t idx = (r * uint64_t(h.live.size())) >> 32;
            int64_t x = h.live[idx];
            int64_t keep = 0;        // bytes of the victim that stay live
            if (!h.segregated()) keep = int64_t((c * uint64_t(h.used.at(x) / h.g)) >> 31) * h.g;
            if (keep == 0) {
                h.dealloc(x);
            } else {
                h.dealloc_partial(x + keep);
            }
            res[i] = x + keep;
        }
    }
}

int64_t copy_state(const Heap& h, int64_t* buf, int64_t cap) {
    std::vector<int64_t> st = h.dump();
    if (buf && int64_t(st.size()) <= cap) std::memcpy(buf, st.data(), st.size() * 8);
    return int64_t(st.size());
}

}  // namespace

extern "C" {

void* orc_heap_new(int algo, int64_t arena, int64_t align) {
    if (!valid_params(algo, arena, align)) return nullptr;
    return new Heap(algo, arena, align);
}
void orc_heap_delete(void* h) { delete static_cast<Heap*>(h); }
int64_t orc_alloc(void* h, int64_t size) { return static_cast<Heap*>(h)->alloc(size); }
int orc_dealloc(void* h, int64_t off) { return static_cast<Heap*>(h)->dealloc(off); }
int orc_dealloc_partial(void* h, int64_t off) {
    return static_cast<Heap*>(h)->dealloc_partial(off);
}
int64_t orc_dump(void* h, int64_t* buf, int64_t cap) {
    return copy_state(*static_cast<Heap*>(h), buf, cap);
}
void orc_stats(void* h, uint64_t* out2) {
    out2[0] = static_cast<Heap*>(h)->examined;
    out2[1] = static_cast<Heap*>(h)->touched;
}
// Replay request i in order on heap h (same driver as orc_replay).
void orc_replay_on(void* h, int64_t n, const int64_t* req, int64_t* res) {
    replay_one(*static_cast<Heap*>(h), n, req, res);
}

// Replay a CSR batch of heaps on `threads` host threads (heaps are split
// longest-first over the threads).  state/state_off may be null; otherwise
// heap i's state is written at state + state_off[i] with capacity
// state_off[i+1]-state_off[i] and its length (in words) to state_len[i].
// stats (may be null) receives per-heap {examined, touched}.
int orc_replay_batch(int64_t H, const int64_t* arena, const int64_t* align,
                     const int32_t* algo, const int64_t* req_off, const int64_t* req,
                     int64_t* res, int64_t* state, const int64_t* state_off,
                     int64_t* state_len, uint64_t* stats, int threads) {
    for (int64_t i = 0; i < H; ++i)
        if (!valid_params(algo[i], arena[i], align[i])) return E_INVAL;
    std::vector<int64_t> order(H);
    for (int64_t i = 0; i < H; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return req_off[a + 1] - req_off[a] > req_off[b + 1] - req_off[b];
    });
    if (threads < 1) threads = 1;
    std::vector<std::vector<int64_t>> part(threads);
    std::vector<int64_t> load(threads, 0);
    for (int64_t i : order) {                 // longest-processing-time first
        int t = int(std::min_element(load.begin(), load.end()) - load.begin());
        part[t].push_back(i);
        load[t] += req_off[i + 1] - req_off[i];
    }
    auto work = [&](int t) {
        for (int64_t i : part[t]) {
            Heap h(algo[i], arena[i], align[i]);
            replay_one(h, req_off[i + 1] - req_off[i], req + req_off[i], res + req_off[i]);
            if (state)
                state_len[i] = copy_state(h, state + state_off[i], state_off[i + 1] - state_off[i]);
            if (stats) { stats[2 * i] = h.examined; stats[2 * i + 1] = h.touched; }
        }
    };
    if (threads == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (int t = 0; t < threads; ++t) th.emplace_back(work, t);
        for (auto& x : th) x.join();
    }
    return 0;
}

}  // extern "C"
