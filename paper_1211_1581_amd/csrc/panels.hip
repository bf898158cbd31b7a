// panels.hip -- y = A x with x staged in LDS by column panels, for matrices
// whose columns scatter over an x far larger than a CU's LDS (Sec. 3.2's
// row-wise product, regrouped so that each gather reads LDS instead of
// missing the vector L1).
//
// Layout (built once per matrix, on request): every row is cut into pieces
// ("virtual rows", one for an empty row) of at most kPiece entries taken with a
// stride (piece j of a row of np pieces holds its entries j, j + np, ...), the
// rows into R ranges of balanced work (merge coordinate, one range per
// kPanelGroups CUs), the columns into panels of W entries of x (64 KB of
// doubles, 112 KB of floats).  A piece's entries in one panel form a segment,
// short because the stride spreads the piece over the row's columns.  Within
// each (range, panel) block the segments are packed into kPanelThreads lanes
// of equal height H (a lane holds whole segments one after another, padding
// where a lane is shorter).  The block is stored chunk by chunk, a chunk being
// U rounds of all lanes (fewer in a block's last chunk), each lane's entries of
// a chunk side by side, so a lane loads them as one vector.  The library keeps
// its own copy of the values in that order and
// per entry one 32-bit word: the column in the panel (bits 0-15), the piece's
// index in its range (bits 16-29), a padding flag (bit 30) and a flag on each
// segment's last entry (bit 31).
//
// The product: kPanelGroups 1024-thread workgroups per range, one per column
// group (the panels holding a quarter of the range's entries), so each range
// reads x once in all.  A workgroup walks its panels in order; thread t sums
// lane t of each block serially (value x LDS slice of x) and, at an entry
// flagged as a segment's last, adds the sum to the piece's accumulator in LDS.
// A piece has one segment per panel, in one lane, so no two additions of one
// panel meet and no barrier is needed between its rounds.  The next panel's
// slice of x is loaded into registers while the current panel is used and
// written to LDS at the switch; two chunks of entries are in flight per
// thread.  At the end each row adds its pieces in order into the group's
// partial vector, and a second kernel adds the groups' parts in group order.
// The order of every addition depends only on the matrix.
#include <algorithm>
#include <atomic>
#include <vector>

#include "internal.h"
#include "scan.h"

namespace spcg {

static std::atomic<int> g_panels{SPCG_PANELS_AUTO};

int panels_mode() { return g_panels.load(std::memory_order_relaxed); }

constexpr int kPanelThreads = 1024;  // = the lanes of a (range, panel) block
constexpr int kPanelMaxRows = 10240;  // virtual rows per range (accumulators in LDS)
constexpr int kPanelGroups = 4;       // column groups: workgroups per range
constexpr int kPanelMaxP = 1024;      // panels
constexpr int kPiece = 32;            // entries per virtual row, at most
constexpr uint32_t kKeyPad = 1u << 30;   // a padding entry: no product
constexpr uint32_t kKeyLast = 1u << 31;  // the last entry of its segment: flush the lane's sum
constexpr uint32_t kKeyRow = 0x3fffu;    // the virtual row field, after the shift by 16
static_assert(kPanelMaxRows <= (1 << 14), "the key's virtual row field has 14 bits");

// One slice of x by value size: 64 KB of doubles (4 16-byte units per thread;
// with 80 KB of accumulators), 112 KB of floats (7 units; 40 KB of
// accumulators).
constexpr int panel_bytes(int esz) { return esz == 8 ? 64 * 1024 : 112 * 1024; }

template <typename T>
constexpr int panel_width() { return panel_bytes((int)sizeof(T)) / (int)sizeof(T); }

// Rounds per chunk (each lane's entries per chunk, two chunks in flight): a
// chunk runs all its rounds, so the short FP64 blocks (lognormal: 4 to 11
// rounds of 1024 lanes) waste fewer with 2, the FP32 blocks (about 35 rounds)
// keep more loads in flight with 4.
template <typename T>
constexpr int panel_rounds() { return sizeof(T) == 8 ? 2 : 4; }

// padding entries after the copy: a lane's vector load in a block's last,
// shorter chunk reaches up to this many entries past the block
constexpr int kPanelPad = 4;

struct PanelDev {
    const int32_t *__restrict__ base;    // [R + 1] first entry of each range
    const int32_t *__restrict__ vstart;  // [n + 1] first virtual row of each row
    const int32_t *__restrict__ range;   // [R + 1] first row of each range
    const int32_t *__restrict__ phase;   // [R][P + 1] entry offset of each panel in its range
    const void *__restrict__ val;        // panel-ordered values
    const uint32_t *__restrict__ key;    // panel column | virtual row in the range << 16 | flags
    void *__restrict__ part;             // [kPanelGroups][n_rows] the groups' partial products
    int P, n_cols, n_rows;
};

// s[b] + ... + s[e - 1] added to part in index order, eight independent LDS
// reads at a time (the lanes past e add +0.0, which leaves a sum that started
// at +0.0 unchanged)
template <typename T>
__device__ __forceinline__ T add_run(T part, const T *s, int b, int e) {
    for (int k = b; k < e; k += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = s[min(k + u, e - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) part += k + u < e ? v[u] : T(0);
    }
    return part;
}

// virtual rows of a row of len entries
__device__ __forceinline__ int pieces(int len) { return len > 0 ? (len + kPiece - 1) / kPiece : 1; }

// the row holding virtual row v: the last i with vstart[i] <= v
__device__ __forceinline__ int row_of(int n, const int32_t *__restrict__ vstart, int v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vstart[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------- analysis --

// Policy SPCG_PANELS_AUTO: the span (last column - first column) of sampled
// rows i = j * stride, j < m (0 for rows of fewer than two entries)
__global__ void __launch_bounds__(kBlock)
k_pan_spans(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t stride, int m,
            int32_t *__restrict__ span) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    const int i = (int)min((int64_t)j * stride, (int64_t)n - 1);
    const int a = rp[i], b = rp[i + 1];
    span[j] = b - a >= 2 ? col[b - 1] - col[a] : 0;
}

__global__ void k_pan_zero(int32_t *flags) {
    if (threadIdx.x == 0) flags[0] = 0;
}

// range[r] = first row i with row_ptr[i] + i >= r * M / R; range[R] = n
__global__ void __launch_bounds__(kBlock)
k_pan_ranges(int n, const int32_t *__restrict__ rp, int R, int64_t M, int32_t *__restrict__ range) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r > R) return;
    if (r == R) {
        range[R] = n;
        return;
    }
    const int64_t target = M * r / R;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if ((int64_t)rp[mid] + mid >= target) hi = mid;
        else lo = mid + 1;
    }
    range[r] = lo;
}

// Virtual rows per row (one for an empty row); flags[0] |= 1 for a row whose
// columns are not strictly increasing
__global__ void __launch_bounds__(kBlock)
k_pan_pieces(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
             int32_t *__restrict__ cnt, int32_t *flags) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int a = rp[i], b = rp[i + 1];
    cnt[i] = pieces(b - a);
    int bad = 0;
    for (int k = a + 1; k < b; ++k) bad |= col[k] <= col[k - 1];
    if (bad) atomicOr(&flags[0], 1);
}

// Virtual row j of a row of np takes the row's entries j, j + np, j + 2 np, ...
// (strided, so every virtual row spreads over the row's columns and its
// segments, its entries in one panel, stay short).  One thread per virtual
// row: its entries per panel (cnt[v * P + p], zeroed before).
__global__ void __launch_bounds__(kBlock)
k_pan_counts(int n, int V, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
             const int32_t *__restrict__ vstart, int W, int P, uint32_t *__restrict__ cnt) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= V) return;
    const int i = row_of(n, vstart, v);
    const int np = vstart[i + 1] - vstart[i];
    uint32_t *c0 = cnt + (size_t)v * P;
    for (int k = rp[i] + (v - vstart[i]); k < rp[i + 1]; k += np) ++c0[col[k] / W];
}

// One wavefront per (range r, panel p) block: the segments (the block's
// virtual rows' entries in the panel, at most kPiece each) are packed into
// kPanelThreads lanes of equal height H (rounds 0..H-1 of each lane); the
// block holds kPanelThreads * H entries.  Lane
// by lane, each lane takes the longest remaining segment that fits its rest
// (H = max(ceil(entries / lanes), longest segment), raised by one until all
// fit; the segments of one length are taken in virtual-row order).  Each
// count cnt[v * P + p] is then replaced by its segment's place: lane | first
// round << 10.  blk_h[r * P + p] = H; flags[0] |= 2 if none fits (never
// expected: from H = entries / lanes + kPiece on every segment fits).
__global__ void __launch_bounds__(64)
k_pan_pack(int P, const int32_t *__restrict__ range, const int32_t *__restrict__ vstart,
           uint32_t *__restrict__ cnt, int32_t *__restrict__ blk_h, int32_t *flags) {
    __shared__ uint32_t take[kPanelMaxRows];           // places, grouped by segment length
    __shared__ int hist[kPiece + 1], off[kPiece + 1], nxt[kPiece + 1];
    const int r = blockIdx.x / P, p = blockIdx.x % P, lane = threadIdx.x;
    const int a = vstart[range[r]], rows = vstart[range[r + 1]] - a;
    uint32_t *cp = cnt + (size_t)a * P + p;
    if (lane <= kPiece) hist[lane] = 0;
    __syncthreads();
    int ent = 0, longest = 0;
    for (int j = lane; j < rows; j += 64) {
        const int c = (int)cp[(size_t)j * P];
        if (c > 0) atomicAdd(&hist[c], 1);
        ent += c;
        longest = max(longest, c);
    }
    for (int o = 32; o > 0; o >>= 1) {
        ent += __shfl_xor(ent, o);
        longest = max(longest, __shfl_xor(longest, o));
    }
    __syncthreads();
    if (lane == 0) {
        int o = 0;
        for (int c = kPiece; c >= 1; --c) {
            off[c] = o;
            o += hist[c];
        }
        int H = ent == 0 ? 0 : max((ent + kPanelThreads - 1) / kPanelThreads, longest);
        bool fits = ent == 0;
        for (int tries = 0; !fits && tries <= kPiece + 1; ++tries, ++H) {
            uint32_t mask = 0;  // bit c - 1: segments of length c remain
            for (int c = 1; c <= kPiece; ++c) {
                nxt[c] = off[c];
                if (hist[c] > 0) mask |= 1u << (c - 1);
            }
            for (int l = 0; l < kPanelThreads && mask; ++l) {
                int cap = H, pos = 0;
                while (cap > 0) {
                    const uint32_t m = mask & (cap >= 32 ? 0xffffffffu : (1u << cap) - 1u);
                    if (!m) break;
                    const int c = 32 - __clz(m);
                    const int idx = nxt[c], end = off[c] + hist[c];
                    const int k = min(cap / c, end - idx);
                    for (int q = 0; q < k; ++q) take[idx + q] = (uint32_t)l | (uint32_t)(pos + q * c) << 10;
                    nxt[c] = idx + k;
                    pos += k * c;
                    cap -= k * c;
                    if (idx + k == end) mask &= ~(1u << (c - 1));
                }
            }
            if (!mask) {
                fits = true;
                break;
            }
        }
        if (!fits) atomicOr(&flags[0], 2);
        blk_h[blockIdx.x] = fits ? H : 0;
        for (int c = 1; c <= kPiece; ++c) nxt[c] = off[c];  // cursors of the placement pass
    }
    __syncthreads();
    // places in virtual-row order, 64 rows at a time: the rows of one length
    // ranked by ballot (lanes of a wavefront run in lockstep; nxt[] is read and
    // advanced by the whole wavefront at once)
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int j0 = 0; j0 < rows; j0 += 64) {
        const int j = j0 + lane;
        const int c = j < rows ? (int)cp[(size_t)j * P] : 0;
        bool pending = c > 0;
        while (true) {
            const unsigned long long pend = __ballot(pending);
            if (!pend) break;
            const int c0 = __shfl(c, __ffsll((long long)pend) - 1);
            const unsigned long long m = __ballot(pending && c == c0);
            const int base = nxt[c0];
            if (pending && c == c0) {
                cp[(size_t)j * P] = take[base + __popcll(m & below)];
                pending = false;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) nxt[c0] = base + __popcll(m);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Per range (one thread each): every panel's first entry in the range and the
// range's entry count (into tot[r]); flags[0] |= 4 if that count overflows int32
__global__ void __launch_bounds__(kBlock)
k_pan_phase(int R, int P, const int32_t *__restrict__ blk_h, int32_t *__restrict__ phase,
            int32_t *__restrict__ tot, int32_t *flags) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= R) return;
    int64_t o = 0;
    for (int p = 0; p < P; ++p) {
        phase[(size_t)r * (P + 1) + p] = (int32_t)min(o, (int64_t)INT32_MAX);
        o += (int64_t)kPanelThreads * blk_h[(size_t)r * P + p];
    }
    phase[(size_t)r * (P + 1) + P] = (int32_t)min(o, (int64_t)INT32_MAX);
    tot[r] = (int32_t)min(o, (int64_t)INT32_MAX);
    if (o > INT32_MAX) atomicOr(&flags[0], 4);
}

// The panel-ordered copy, one thread per virtual row: entry q of a segment
// placed at (lane l, first round h0) goes to the block's entry
// (h0 + q) * kPanelThreads + l, with key panel column | virtual row in the
// range << 16 | kKeyLast on the segment's last entry
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_pan_scatter(int n, int V, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
              const T *__restrict__ vals, int W, int P, int R, const int32_t *__restrict__ range,
              const int32_t *__restrict__ vstart, const uint32_t *__restrict__ place,
              const int32_t *__restrict__ phase, const int32_t *__restrict__ rbase,
              T *__restrict__ pval, uint32_t *__restrict__ pkey) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= V) return;
    const int i = row_of(n, vstart, v);
    int lo = 0, hi = R - 1;  // the last range r with range[r] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (range[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const int r = lo, vl = v - vstart[range[r]], np = vstart[i + 1] - vstart[i], b = rp[i + 1];
    constexpr int U = panel_rounds<T>();
    int prev = -1, blk = 0, H = 0, lane = 0, h = 0;
    for (int k = rp[i] + (v - vstart[i]); k < b; k += np, ++h) {
        const int c = col[k], p = c / W;
        if (p != prev) {
            const uint32_t pl = place[(size_t)v * P + p];
            const size_t ph = (size_t)r * (P + 1) + p;
            blk = rbase[r] + phase[ph];
            H = (phase[ph + 1] - phase[ph]) / kPanelThreads;
            lane = (int)(pl & (kPanelThreads - 1));
            h = (int)(pl >> 10);
            prev = p;
        }
        // round h of the lane: chunk h / U holds rc = min(U, H - its first round)
        // rounds, each lane's rc entries side by side
        const int ch = h / U, rc = min(U, H - ch * U);
        const int pos = blk + ch * U * kPanelThreads + lane * rc + (h - ch * U);
        const bool last = k + np >= b || col[k + np] / W != p;
        pval[pos] = vals[k];
        pkey[pos] = (uint32_t)(c - p * W) | (uint32_t)vl << 16 | (last ? kKeyLast : 0u);
    }
}

// ---------------------------------------------------------------- product --

// Slice p of x (elements [p W, min((p + 1) W, n_cols))) as 16-byte units,
// panel_bytes / 16 / kPanelThreads per thread; elements past n_cols are zero.
// Every unit is one 16-byte load with no branch: a unit that reaches past
// n_cols reads the last E elements of x instead (n_cols >= E; an address that
// is not 16-byte aligned is served by the unaligned access mode), and the
// store shifts its elements into place.
template <typename T>
struct Slice {
    static constexpr int E = 16 / sizeof(T);  // elements per unit
    static constexpr int U = panel_bytes((int)sizeof(T)) / 16 / kPanelThreads;
    uint4 u[U];
    int p;
    __device__ __forceinline__ void load(const T *__restrict__ x, int n_cols, int p_) {
        constexpr int W = panel_width<T>();
        p = p_;
#pragma unroll
        for (int v = 0; v < U; ++v) {
            const int e = p * W + (threadIdx.x + v * kPanelThreads) * E;
            __builtin_memcpy(&u[v], x + min(e, n_cols - E), 16);
        }
    }
    __device__ __forceinline__ void store(T *xs, int n_cols) const {
        constexpr int W = panel_width<T>();
#pragma unroll
        for (int v = 0; v < U; ++v) {
            const int e = p * W + (threadIdx.x + v * kPanelThreads) * E;
            const int sh = e - min(e, n_cols - E);  // the unit's first element in the load
            T L[E], o[E];
            __builtin_memcpy(L, &u[v], 16);
#pragma unroll
            for (int q = 0; q < E; ++q) {
                T t = L[0];
#pragma unroll
                for (int k = 1; k < E; ++k) t = q + sh == k ? L[k] : t;
                o[q] = e + q < n_cols ? t : T(0);
            }
            __builtin_memcpy(xs + (threadIdx.x + v * kPanelThreads) * E, o, 16);
        }
    }
};

// A thread's entries of a chunk in registers: with U rounds per chunk and rc
// of them in chunk c (rc = U but in a block's last chunk), round u of lane t
// is the block's entry c U kPanelThreads + t rc + u
template <typename T>
struct Entries {
    T v[panel_rounds<T>()];
    uint32_t k[panel_rounds<T>()];
};

template <typename T>
__global__ void __launch_bounds__(kPanelThreads)
k_spmv_panels(PanelDev D, const T *__restrict__ x) {
    constexpr int W = panel_width<T>();
    constexpr int kPanelU = panel_rounds<T>(), kPanelChunk = kPanelThreads * kPanelU;
    __shared__ __align__(16) T xs[W];      // the panel's slice of x
    __shared__ T vacc[kPanelMaxRows];      // every virtual row's running sum
    __shared__ int ph[kPanelMaxP + 1];
    const int tid = threadIdx.x;
    // workgroup -> (range r, column group grp)
    const int r = blockIdx.x / kPanelGroups, grp = blockIdx.x % kPanelGroups;
    const int a = D.range[r], rows = D.range[r + 1] - a;
    if (rows <= 0) return;  // uniform
    const int va = D.vstart[a], vrows = D.vstart[a + rows] - va;
    const int PT = D.P;
    const int base = D.base[r];
    const T *__restrict__ val = (const T *)D.val + base;
    const uint32_t *__restrict__ key = D.key + base;
    for (int p = tid; p <= PT; p += kPanelThreads) ph[p] = D.phase[(size_t)r * (PT + 1) + p];
    for (int j = tid; j < vrows; j += kPanelThreads) vacc[j] = T(0);
    __syncthreads();
    // the group's panels [p0, P): a quarter of the range's entries (the first
    // panel p with ph[p] >= g / kPanelGroups of them starts group g)
    auto split = [&](int g) {
        if (g >= kPanelGroups) return PT;
        const int64_t t = (int64_t)ph[PT] * g / kPanelGroups;
        int lo = 0, hi = PT;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ph[mid] >= t) hi = mid;
            else lo = mid + 1;
        }
        return lo;
    };
    const int p0 = grp == 0 ? 0 : split(grp), P = split(grp + 1);

    auto next_panel = [&](int p) {  // the first non-empty panel after p (P if none)
        ++p;
        while (p < P && ph[p + 1] == ph[p]) ++p;
        return p;
    };
    // chunks are walked in order: panel by panel, kPanelChunk entries at a
    // time; past the group's last panel the position stays at P
    auto advance = [&](int &p, int &c) {
        if (p >= P) return;
        c += kPanelChunk;
        if (c >= ph[p + 1] - ph[p]) {
            c = 0;
            p = next_panel(p);
        }
    };
    // a lane's kPanelU entries of a chunk lie side by side (rc of them in a
    // block's last chunk of rc rounds; the load then also takes the next
    // lane's, which the round mask discards): one vector of values and one of
    // keys.  Issued even past the last chunk (then of the range's last
    // entries), so the number of loads in flight after each set is the same
    // on every path
    typedef T vals_t __attribute__((ext_vector_type(kPanelU)));
    typedef uint32_t keys_t __attribute__((ext_vector_type(kPanelU)));
    auto fetch = [&](Entries<T> &E, int p, int c) {
        const int rc = p < P ? min(kPanelU, (ph[p + 1] - ph[p] - c) / kPanelThreads) : 0;
        const int e = p < P ? ph[p] + c + tid * rc : ph[P] - kPanelU;
        const vals_t vv = __builtin_nontemporal_load((const vals_t *)(val + e));
        const keys_t kk = __builtin_nontemporal_load((const keys_t *)(key + e));
#pragma unroll
        for (int u = 0; u < kPanelU; ++u) {
            E.v[u] = vv[u];
            E.k[u] = kk[u];
        }
    };

    const int first = next_panel(p0 - 1);
    if (first < P) {
        // the first panel's slice now, the next panel's in flight
        {
            Slice<T> s0;
            s0.load(x, D.n_cols, first);
            s0.store(xs, D.n_cols);
        }
        Slice<T> sn;
        int pnext = next_panel(first);
        sn.load(x, D.n_cols, pnext < P ? pnext : first);  // (a spare load if there is none)
        // two chunks of entries in flight: A and B take turns
        int pf = first, cf = 0;  // the next chunk to fetch
        Entries<T> A, B;
        fetch(A, pf, cf);
        advance(pf, cf);
        fetch(B, pf, cf);
        advance(pf, cf);
        __syncthreads();
        int pc = first, cc = 0;  // the chunk being summed
        T acc = T(0);            // the lane's sum of its current segment
        auto step = [&](Entries<T> &E) {
            if (pc < P && cc == 0 && pc != first) {
                // a new panel: every wavefront is done with the last slice; the
                // new one arrived during the last panel
                __syncthreads();
                sn.store(xs, D.n_cols);
                pnext = next_panel(pc);
                sn.load(x, D.n_cols, pnext < P ? pnext : pc);
                __syncthreads();
            }
            // products (a padding entry, or a round past the block: none) and
            // the lane's segments, entry by entry: at a segment's last entry its
            // sum goes to its virtual row (a virtual row has one segment per
            // panel, so no two lanes add to one row within a panel).  E is
            // consumed whole before it is refilled with the chunk after the
            // other set's, so the refill lands in E's own registers (values
            // still live across the refill made the compiler load into other
            // registers and copy them at the loop's end, waiting for the loads)
            const int rounds = pc < P ? min(kPanelU, (ph[pc + 1] - ph[pc] - cc) / kPanelThreads) : 0;
#pragma unroll
            for (int u = 0; u < kPanelU; ++u) {
                const uint32_t k = u < rounds ? E.k[u] : kKeyPad;
                const T t = E.v[u] * xs[k & 0xffffu];
                acc += (k & kKeyPad) ? T(0) : t;
                if (k & kKeyLast) {
                    vacc[(k >> 16) & kKeyRow] += acc;
                    acc = T(0);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            fetch(E, pf, cf);
            advance(pf, cf);
            advance(pc, cc);
        };
        // A and B on every trip (B past the last chunk sums nothing): with no
        // path that loops back after A alone, the compiler sees the other
        // set's loads as the newer ones at each step and waits only for the
        // set it sums (an exit between the two made it wait for every load)
        do {
            step(A);
            step(B);
        } while (pc < P);
    }
    // every row of the range: the group's part, its pieces' sums in order
    __syncthreads();
    T *__restrict__ yp = (T *)D.part + (size_t)grp * D.n_rows;
    for (int i = tid; i < rows; i += kPanelThreads)
        yp[a + i] = add_run(T(0), vacc, D.vstart[a + i] - va, D.vstart[a + i + 1] - va);
}

// y_i = the column groups' parts of row i added in group order
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_pan_combine(int n, const T *__restrict__ part, T *__restrict__ y) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    T s = part[i];
#pragma unroll
    for (int g = 1; g < kPanelGroups; ++g) s += part[(size_t)g * n + i];
    y[i] = s;
}

// ------------------------------------------------------------------ host --

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

int build_panels(spcg_csr *h, hipStream_t s) {
    const int n = h->n_rows;
    if (n == 0 || h->nnz == 0) return SPCG_OK;
    const int esz = h->dtype == SPCG_F64 ? 8 : 4;
    const int W = panel_bytes(esz) / esz;
    const int64_t P64 = ((int64_t)h->n_cols + W - 1) / W;
    if (P64 > kPanelMaxP || h->n_cols < 4) return SPCG_OK;  // x too wide for the panel table, or
                                                              // narrower than a 16-byte unit: not built
    const int P = (int)std::max<int64_t>(P64, 1);
    const int R = std::max(1, std::min(device_cus() / kPanelGroups, n));  // one range per kPanelGroups CUs
    uint32_t *cnt = nullptr;  // analysis only: counts, then places, per (virtual row, panel)
    int32_t *pcs = nullptr, *sums = nullptr, *blk = nullptr;
    auto release = [&]() {
        if (cnt) (void)hipFree(cnt);
        for (int32_t *q : {pcs, sums, blk})
            if (q) (void)hipFree(q);
        cnt = nullptr;
        pcs = sums = blk = nullptr;
    };
    auto fail = [&](hipError_t e, const char *what) {
        release();
        return hip_status(e, what);
    };
    auto done = [&]() {  // not built: every panel array goes, the product keeps its default path
        release();
        for (int32_t *q : {h->pan_range, h->pan_vstart, h->pan_phase, h->pan_base})
            if (q) (void)hipFree(q);
        for (void *q : {(void *)h->pan_key, h->pan_val, h->pan_part})
            if (q) (void)hipFree(q);
        h->pan_range = h->pan_vstart = h->pan_phase = h->pan_base = nullptr;
        h->pan_key = nullptr;
        h->pan_val = h->pan_part = nullptr;
        return SPCG_OK;
    };
    hipError_t e;
    int32_t *hp = (int32_t *)h->h_pinned;
    // ranges of rows, then the virtual rows of every row (vstart[n] = all of
    // them) and the sorted-columns check
    if ((e = hipMalloc(&h->pan_range, sizeof(int32_t) * ((size_t)R + 1))) != hipSuccess ||
        (e = hipMalloc(&h->pan_vstart, sizeof(int32_t) * ((size_t)n + 1))) != hipSuccess ||
        (e = hipMalloc(&pcs, sizeof(int32_t) * (size_t)n)) != hipSuccess ||
        (e = hipMalloc(&sums, sizeof(int32_t) * (size_t)scan_sums_slots(n))) != hipSuccess)
        return fail(e, "hipMalloc(panel ranges)");
    hipLaunchKernelGGL(k_pan_zero, dim3(1), dim3(64), 0, s, h->flags);
    hipLaunchKernelGGL(k_pan_ranges, dim3((R + kBlock) / kBlock), dim3(kBlock), 0, s, n, h->row_ptr, R,
                       (int64_t)h->nnz + n, h->pan_range);
    hipLaunchKernelGGL(k_pan_pieces, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, h->row_ptr, h->col,
                       pcs, h->flags);
    exclusive_scan(n, pcs, sums, h->pan_vstart, s);
    std::vector<int32_t> rr((size_t)R + 1), vs((size_t)n + 1);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(rr.data(), h->pan_range, sizeof(int32_t) * (R + 1), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(vs.data(), h->pan_vstart, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipMemcpyAsync(hp, h->flags, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e, "panel ranges");
    if (hp[0] != 0) return done();  // a row with unsorted columns
    for (int32_t *q : {pcs, sums}) (void)hipFree(q);
    pcs = sums = nullptr;
    for (int r = 0; r < R; ++r)
        if (vs[rr[r + 1]] - vs[rr[r]] > kPanelMaxRows) return done();  // too many for a workgroup
    const int V = vs[n];
    // entries per (virtual row, panel), then the segments packed into lanes
    // (each count replaced by its place) and the blocks' heights, then the
    // panels' first entries and each range's entry count (into pan_base for now)
    if ((e = hipMalloc(&cnt, sizeof(uint32_t) * (size_t)V * P)) != hipSuccess ||
        (e = hipMalloc(&blk, sizeof(int32_t) * (size_t)R * P)) != hipSuccess ||
        (e = hipMalloc(&h->pan_phase, sizeof(int32_t) * (size_t)R * (P + 1))) != hipSuccess ||
        (e = hipMalloc(&h->pan_base, sizeof(int32_t) * ((size_t)R + 1))) != hipSuccess ||
        (e = hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (size_t)V * P, s)) != hipSuccess)
        return fail(e, "hipMalloc(panel layout)");
    hipLaunchKernelGGL(k_pan_counts, dim3((V + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, V, h->row_ptr,
                       h->col, (const int32_t *)h->pan_vstart, W, P, cnt);
    hipLaunchKernelGGL(k_pan_pack, dim3(R * P), dim3(64), 0, s, P, (const int32_t *)h->pan_range,
                       (const int32_t *)h->pan_vstart, cnt, blk, h->flags);
    hipLaunchKernelGGL(k_pan_phase, dim3((R + kBlock - 1) / kBlock), dim3(kBlock), 0, s, R, P,
                       (const int32_t *)blk, h->pan_phase, h->pan_base, h->flags);
    std::vector<int32_t> tot((size_t)R);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(tot.data(), h->pan_base, sizeof(int32_t) * R, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(hp, h->flags, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e, "panel layout");
    if (hp[0] != 0) return done();  // no packing found, or a range beyond int32 entries
    std::vector<int32_t> rb((size_t)R + 1, 0);
    int64_t total = 0;
    for (int r = 0; r < R; ++r) {
        rb[r] = (int32_t)total;
        total += tot[r];
        if (total > INT32_MAX) return done();  // too many entries with the padding
    }
    // blocks so sparse that their lanes are mostly padding: the row blocks do better
    if (total > 2 * (int64_t)h->nnz + (int64_t(1) << 24)) return done();
    rb[R] = (int32_t)total;
    if ((e = hipMemcpyAsync(h->pan_base, rb.data(), sizeof(int32_t) * ((size_t)R + 1), hipMemcpyHostToDevice,
                            s)) != hipSuccess ||
        (e = hipMalloc(&h->pan_val, (size_t)esz * (total + kPanelPad))) != hipSuccess ||
        (e = hipMalloc(&h->pan_key, sizeof(uint32_t) * (total + kPanelPad))) != hipSuccess ||
        (e = hipMalloc(&h->pan_part, (size_t)esz * kPanelGroups * n)) != hipSuccess ||
        (!h->pan_done && (e = hipEventCreateWithFlags(&h->pan_done, hipEventDisableTiming)) != hipSuccess) ||
        (e = hipMemsetAsync(h->pan_val, 0, (size_t)esz * (total + kPanelPad), s)) != hipSuccess ||
        (e = hipMemsetD32Async((hipDeviceptr_t)h->pan_key, (int)kKeyPad, (size_t)(total + kPanelPad), s)) !=
            hipSuccess)
        return fail(e, "hipMalloc(panels)");
    if (esz == 8)
        hipLaunchKernelGGL(k_pan_scatter<double>, dim3((V + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, V,
                           h->row_ptr, h->col, (const double *)h->vals, W, P, R, (const int32_t *)h->pan_range,
                           (const int32_t *)h->pan_vstart, (const uint32_t *)cnt,
                           (const int32_t *)h->pan_phase, (const int32_t *)h->pan_base, (double *)h->pan_val,
                           h->pan_key);
    else
        hipLaunchKernelGGL(k_pan_scatter<float>, dim3((V + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, V,
                           h->row_ptr, h->col, (const float *)h->vals, W, P, R, (const int32_t *)h->pan_range,
                           (const int32_t *)h->pan_vstart, (const uint32_t *)cnt,
                           (const int32_t *)h->pan_phase, (const int32_t *)h->pan_base, (float *)h->pan_val,
                           h->pan_key);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e, "k_pan_scatter");
    release();
    h->pan_P = P;
    h->pan_R = R;
    h->pan_W = W;
    h->pan_entries = total;
    h->has_panels = true;
    return SPCG_OK;
}

bool use_panels(const spcg_csr *A) { return A->has_panels && panels_mode() != SPCG_PANELS_OFF; }

// Policy SPCG_PANELS_AUTO: panels pay for matrices whose rows gather from
// across a wide x: at least kAutoRows rows, kAutoLen entries per row on
// average, and sampled rows spanning more than a quarter of the columns at
// the median (the lognormal input: 96 %; a band or a stencil: a few per cent
// or less, and their rows are short or local, so x comes from the caches)
constexpr int kAutoRows = 1 << 16;
constexpr int kAutoLen = 16;
constexpr int kAutoSamples = 4096;

int panels_pay(const spcg_csr *h, hipStream_t s, bool *pay) {
    *pay = false;
    const int n = h->n_rows;
    if (n < kAutoRows || h->nnz < (int64_t)kAutoLen * n) return SPCG_OK;
    const int m = std::min(n, kAutoSamples);
    const int64_t stride = n / m;
    int32_t *d = nullptr;
    std::vector<int32_t> span((size_t)m);
    hipError_t e;
    if ((e = hipMalloc(&d, sizeof(int32_t) * m)) != hipSuccess) return hip_status(e, "hipMalloc(panel spans)");
    hipLaunchKernelGGL(k_pan_spans, dim3((m + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, h->row_ptr, h->col,
                       stride, m, d);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(span.data(), d, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        (void)hipFree(d);
        return hip_status(e, "panel spans");
    }
    (void)hipFree(d);
    std::nth_element(span.begin(), span.begin() + m / 2, span.end());
    *pay = (int64_t)span[m / 2] * 4 > (int64_t)h->n_cols;
    return SPCG_OK;
}

template <typename T>
int launch_spmv_panels(const spcg_csr *A, const T *x, T *y, hipStream_t s) {
    // products share the handle's partial vectors: one on another stream than
    // the last waits for the last one's completion (on one stream, the order of
    // the stream already does)
    spcg_csr *H = const_cast<spcg_csr *>(A);
    std::lock_guard<std::mutex> lock(H->pan_mu);
    if (H->pan_any && H->pan_last != s) SPCG_TRY(hipStreamWaitEvent(s, H->pan_done, 0));
    const PanelDev D{A->pan_base, A->pan_vstart, A->pan_range, A->pan_phase, A->pan_val,
                     A->pan_key, A->pan_part, A->pan_P, A->n_cols, A->n_rows};
    hipLaunchKernelGGL(k_spmv_panels<T>, dim3(A->pan_R * kPanelGroups), dim3(kPanelThreads), 0, s, D, x);
    hipLaunchKernelGGL(k_pan_combine<T>, dim3((A->n_rows + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       A->n_rows, (const T *)A->pan_part, y);
    SPCG_LAUNCH_CHECK("k_spmv_panels");
    SPCG_TRY(hipEventRecord(H->pan_done, s));
    H->pan_last = s;
    H->pan_any = true;
    return SPCG_OK;
}

template int launch_spmv_panels<double>(const spcg_csr *, const double *, double *, hipStream_t);
template int launch_spmv_panels<float>(const spcg_csr *, const float *, float *, hipStream_t);

}  // namespace spcg

extern "C" {

int spcg_column_panels(int mode) {
    if (mode < 0) return spcg::g_panels.load();
    if (mode > SPCG_PANELS_AUTO) return SPCG_INVALID_ARG;
    return spcg::g_panels.exchange(mode);
}

int spcg_csr_panel_info(spcg_csr_t A, int64_t *n_ranges, int64_t *n_panels, int64_t *n_entries) {
    if (!A || !A->has_panels) return SPCG_INVALID_ARG;
    if (n_ranges) *n_ranges = A->pan_R;
    if (n_panels) *n_panels = A->pan_P;
    if (n_entries) *n_entries = A->pan_entries;
    return SPCG_OK;
}

}  // extern "C"
