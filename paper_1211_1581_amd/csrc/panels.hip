// panels.hip -- y = A x with x staged in LDS by column panels, for matrices
// whose columns scatter over an x far larger than a CU's LDS (Sec. 3.2's
// row-wise product, regrouped so that each gather reads LDS instead of
// missing the vector L1).
//
// Layout (built once per matrix, on request): every row is cut into pieces of
// at most kPiece consecutive entries ("virtual rows", one for an empty row), the
// rows into R ranges of balanced work (merge coordinate, one range per
// kPanelGroups CUs), the columns into panels of W entries of x (48 KB of
// doubles, 112 KB of floats).  The library keeps its own copy of the values,
// ordered by range, then panel, then virtual row, then column, and per entry
// one 32-bit word: the column in the panel (low 16 bits) and the virtual row's
// index in its range (high 16).  A virtual row's entries in one panel form a
// segment (rows hold sorted columns); within each (range, panel) block no
// segment crosses a multiple of 64 entries: where one would, padding entries
// (value 0, virtual row 0xFFFF) fill the rest of the 64.
//
// The product: kPanelGroups 1024-thread workgroups per range, one per column
// group (a contiguous quarter of the panels), so each range reads x once in
// all.  A workgroup walks its panels in order; each of its wavefronts takes
// 256 of every 4096 entries of a panel's block, in rounds of 64: products
// (value x LDS slice of x), a segmented scan across the lanes by DPP moves (a
// fixed tree in each segment), and each segment's sum added to its virtual
// row's accumulator in LDS.  A virtual row has one segment per panel, so the additions of one
// panel never meet, and no barrier is needed between its rounds.  The next
// panel's slice of x is loaded into registers while the current panel is used
// and written to LDS at the switch; two chunks of entries are in flight per
// wavefront.  At the end each row adds its pieces in order into the group's
// partial vector, and a second kernel adds the groups' parts in group order.
// The order of every addition depends only on the matrix.
#include <algorithm>
#include <atomic>
#include <vector>

#include "internal.h"
#include "scan.h"

namespace spcg {

static std::atomic<int> g_panels{SPCG_PANELS_OFF};

int panels_mode() { return g_panels.load(std::memory_order_relaxed); }

constexpr int kPanelThreads = 1024;
constexpr int kPanelMaxRows = 10240;    // virtual rows per range (accumulators in LDS)
constexpr int kPanelGroups = 4;         // column groups: workgroups per range
constexpr int kPanelU = 4;              // entries per thread and chunk (rounds of 64 per wavefront)
constexpr int kPanelChunk = kPanelThreads * kPanelU;
constexpr int kPanelMaxP = 1024;        // panels
constexpr int kPiece = 32;              // entries per virtual row (at most one lane round)
constexpr uint32_t kPadRow = 0xFFFFu;   // the virtual row of a padding entry

// One slice of x by value size: 48 KB of doubles (3 16-byte units per thread;
// with 80 KB of accumulators), 112 KB of floats (7 units; 40 KB of
// accumulators), the sizes measured fastest on the lognormal matrix.
constexpr int panel_bytes(int esz) { return esz == 8 ? 48 * 1024 : 112 * 1024; }

template <typename T>
constexpr int panel_width() { return panel_bytes((int)sizeof(T)) / (int)sizeof(T); }

struct PanelDev {
    const int32_t *__restrict__ base;    // [R + 1] first entry of each range
    const int32_t *__restrict__ vstart;  // [n + 1] first virtual row of each row
    const int32_t *__restrict__ range;   // [R + 1] first row of each range
    const int32_t *__restrict__ phase;   // [R][P + 1] entry offset of each panel in its range
    const void *__restrict__ val;        // [nnz] panel-ordered values
    const uint32_t *__restrict__ key;    // [nnz] panel column | virtual row in the range << 16
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

// ------------------------------------------------------------- analysis --

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

// Virtual rows per row (pieces of at most kPiece entries, one for an empty row)
__global__ void __launch_bounds__(kBlock)
k_pan_pieces(int n, const int32_t *__restrict__ rp, int32_t *__restrict__ cnt) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) cnt[i] = pieces(rp[i + 1] - rp[i]);
}

// Per virtual row: entries in each panel (cnt[v * P + p]); flags[0] |= 1 for a
// row whose columns are not strictly increasing
__global__ void __launch_bounds__(kBlock)
k_pan_counts(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
             const int32_t *__restrict__ vstart, int W, int P, uint16_t *__restrict__ cnt,
             int32_t *flags) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int a = rp[i], b = rp[i + 1], v0 = vstart[i];
    uint16_t *c0 = cnt + (size_t)v0 * P;
    for (int q = 0; q < pieces(b - a) * P; ++q) c0[q] = 0;
    int prev = -1, bad = 0;
    for (int k = a; k < b; ++k) {
        const int cc = col[k];
        bad |= cc <= prev;
        prev = cc;
        uint16_t *c = cnt + ((size_t)v0 + (k - a) / kPiece) * P + cc / W;
        *c = (uint16_t)(*c + 1);
    }
    if (bad) atomicOr(&flags[0], 1);
}

// One workgroup per range, one thread per panel: the start of every virtual
// row's segment in the panel's block (uint16, padded so that no segment crosses
// a multiple of 64), then the start of every panel in the range (a scan over the
// panels) and the range's entry count (tot[r]).  flags[0] |= 2 if a block holds
// 65536 entries or more.
__global__ void __launch_bounds__(kPanelThreads)
k_pan_layout(int P, const int32_t *__restrict__ range, const int32_t *__restrict__ vstart,
             const uint16_t *__restrict__ cnt, uint16_t *__restrict__ seg,
             int32_t *__restrict__ phase, int32_t *__restrict__ tot, int32_t *flags) {
    __shared__ int sh[kPanelThreads];
    const int r = blockIdx.x, p = threadIdx.x;
    const int a = vstart[range[r]], rows = vstart[range[r + 1]] - a;  // the range's virtual rows
    int pos = 0;
    if (p < P) {
        uint16_t *sp = seg + (size_t)P * (a + r) + (size_t)p * (rows + 1);
        for (int j = 0; j < rows; ++j) {
            const int c = cnt[(size_t)(a + j) * P + p];
            if (c > 0 && (pos & 63) + c > 64) pos = (pos + 63) & ~63;
            sp[j] = (uint16_t)min(pos, 65535);
            pos += c;
        }
        sp[rows] = (uint16_t)min(pos, 65535);
        if (pos > 65535) atomicOr(&flags[0], 2);
    }
    sh[p] = pos;
    __syncthreads();
    for (int o = 1; o < kPanelThreads; o <<= 1) {  // inclusive scan of the block sizes
        const int t = p >= o ? sh[p - o] : 0;
        __syncthreads();
        sh[p] += t;
        __syncthreads();
    }
    if (p < P) phase[(size_t)r * (P + 1) + p] = sh[p] - pos;
    if (p == 0) {
        phase[(size_t)r * (P + 1) + P] = sh[kPanelThreads - 1];
        tot[r] = sh[kPanelThreads - 1];
    }
}

// The panel-ordered copy: values and keys (panel column | virtual row << 16)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_pan_scatter(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
              const T *__restrict__ vals, int W, int P, int R, const int32_t *__restrict__ range,
              const int32_t *__restrict__ vstart, const uint16_t *__restrict__ seg,
              const int32_t *__restrict__ phase, const int32_t *__restrict__ rbase,
              T *__restrict__ pval, uint32_t *__restrict__ pkey) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = R;  // the last range r with range[r] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (range[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const int r = lo, va = vstart[range[r]], vrows = vstart[range[r + 1]] - va;
    const uint16_t *sr = seg + (size_t)P * (va + r);
    const int base = rbase[r], a = rp[i], v0 = vstart[i] - va;
    int prev = -1, pos = 0;
    for (int k = a; k < rp[i + 1]; ++k) {
        const int c = col[k];
        const int p = c / W, v = v0 + (k - a) / kPiece;
        const int key = v * P + p;  // (piece, panel) changes together
        if (key != prev) {
            pos = base + phase[(size_t)r * (P + 1) + p] + sr[(size_t)p * (vrows + 1) + v];
            prev = key;
        }
        pval[pos] = vals[k];
        pkey[pos] = (uint32_t)(c - p * W) | (uint32_t)v << 16;
        ++pos;
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

// A wavefront's share of a chunk in registers: round u, lane l holds entry
// 256 w + 64 u + l of the chunk (w the wavefront)
template <typename T>
struct Entries {
    T v[kPanelU];
    uint32_t k[kPanelU];
};

// v moved across lanes by DPP control CTRL (a VALU operand modifier, no LDS
// round trip) in the rows of 16 lanes that ROWS selects; lanes of other rows,
// and lanes whose source leaves the row, read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp0(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp0(float v) {
    return __int_as_float(dpp0<CTRL, ROWS>(__float_as_int(v)));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp0(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp0<CTRL, ROWS>((int)b), hi = dpp0<CTRL, ROWS>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int kDppRowShr = 0x110;   // + n: lane l <- lane l - n within its row of 16
constexpr int kDppWaveShr1 = 0x138;  // lane l <- lane l - 1 across the wavefront
constexpr int kDppBcast15 = 0x142;   // rows 1 and 3 <- lanes 15 and 47 (row mask 0xA)
constexpr int kDppBcast31 = 0x143;   // rows 2 and 3 <- lane 31 (row mask 0xC)

// Inclusive scan of s over each segment of lanes [start, lane] (a segment
// spans at most 32 lanes, so at most three rows of 16): prefix sums inside the
// rows by four row shifts, then the rows' carries, rows 1 and 3 from lanes 15
// and 47 and rows 2 and 3 from lane 31 (which holds its segment's sum from the
// start by then).  Every lane runs every step; a fixed tree per segment.
template <typename T>
__device__ __forceinline__ T segmented_scan(T s, int lane, int start) {
    T t;
    t = dpp0<kDppRowShr + 1, 0xF>(s);
    if (lane - 1 >= start && (lane & 15) >= 1) s += t;
    t = dpp0<kDppRowShr + 2, 0xF>(s);
    if (lane - 2 >= start && (lane & 15) >= 2) s += t;
    t = dpp0<kDppRowShr + 4, 0xF>(s);
    if (lane - 4 >= start && (lane & 15) >= 4) s += t;
    t = dpp0<kDppRowShr + 8, 0xF>(s);
    if (lane - 8 >= start && (lane & 15) >= 8) s += t;
    t = dpp0<kDppBcast15, 0xA>(s);
    if (((lane >> 4) & 1) && start < (lane & ~15)) s += t;
    t = dpp0<kDppBcast31, 0xC>(s);
    if (lane >= 32 && start < 32) s += t;
    return s;
}

template <typename T>
__global__ void __launch_bounds__(kPanelThreads)
k_spmv_panels(PanelDev D, const T *__restrict__ x) {
    constexpr int W = panel_width<T>();
    __shared__ __align__(16) T xs[W];      // the panel's slice of x; at the end the pieces' sums
    __shared__ T vacc[kPanelMaxRows];      // every virtual row's running sum
    __shared__ int ph[kPanelMaxP + 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wbase = (tid >> 6) * (kPanelChunk / (kPanelThreads / 64));  // the wavefront's entries
    const unsigned long long below = (1ull << lane) - 1ull;
    // workgroup -> (range r, column group grp); the group walks panels [p0, P)
    const int r = blockIdx.x / kPanelGroups, grp = blockIdx.x % kPanelGroups;
    const int a = D.range[r], rows = D.range[r + 1] - a;
    if (rows <= 0) return;  // uniform
    const int va = D.vstart[a], vrows = D.vstart[a + rows] - va;
    const int PT = D.P, per = (PT + kPanelGroups - 1) / kPanelGroups;
    const int p0 = min(grp * per, PT), P = min(p0 + per, PT);
    const int base = D.base[r];
    const T *__restrict__ val = (const T *)D.val + base;
    const uint32_t *__restrict__ key = D.key + base;
    for (int p = tid; p <= PT; p += kPanelThreads) ph[p] = D.phase[(size_t)r * (PT + 1) + p];
    for (int j = tid; j < vrows; j += kPanelThreads) vacc[j] = T(0);
    __syncthreads();

    auto next_panel = [&](int p) {  // the first non-empty panel after p (P if none)
        ++p;
        while (p < P && ph[p + 1] == ph[p]) ++p;
        return p;
    };
    // chunks are walked in order: panel by panel, kPanelChunk entries at a time
    auto advance = [&](int &p, int &c) {
        c += kPanelChunk;
        if (c >= ph[p + 1] - ph[p]) {
            c = 0;
            p = next_panel(p);
        }
    };
    // issued even past the last chunk (then of the range's last entry), so the
    // number of loads in flight after each set is the same on every path
    auto fetch = [&](Entries<T> &E, int p, int c) {
        const int e0 = p < P ? ph[p] + c : ph[P] - 1, last = ph[min(p + 1, P)] - 1;
#pragma unroll
        for (int u = 0; u < kPanelU; ++u) {
            const int e = min(e0 + wbase + 64 * u + lane, last);
            E.v[u] = __builtin_nontemporal_load(val + e);
            E.k[u] = __builtin_nontemporal_load(key + e);
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
        auto step = [&](Entries<T> &E) {
            if (cc == 0 && pc != first) {
                // a new panel: every wavefront is done with the last slice; the
                // new one arrived during the last panel
                __syncthreads();
                sn.store(xs, D.n_cols);
                pnext = next_panel(pc);
                sn.load(x, D.n_cols, pnext < P ? pnext : pc);
                __syncthreads();
            }
            // products and virtual rows (padding and entries past the chunk: row
            // kPadRow, product 0), then E refilled with the chunk after the other
            // set's (kept after the products, so the refill lands in E's own
            // registers instead of copies that wait for every load in flight)
            const int cnt = min(kPanelChunk, ph[pc + 1] - ph[pc] - cc);
            T pr[kPanelU];
            int id[kPanelU];
#pragma unroll
            for (int u = 0; u < kPanelU; ++u) {
                const bool in = wbase + 64 * u + lane < cnt;
                id[u] = in ? (int)(E.k[u] >> 16) : (int)kPadRow;
                const T t = E.v[u] * xs[E.k[u] & 0xffffu];
                pr[u] = id[u] != (int)kPadRow ? t : T(0);
            }
            __builtin_amdgcn_sched_barrier(0);
            fetch(E, pf, cf);
            advance(pf, cf);
            // per round: a segmented scan (segments of at most kPiece lanes), then
            // each segment's last lane adds the sum to its virtual row
#pragma unroll
            for (int u = 0; u < kPanelU; ++u) {
                const int prev = dpp0<kDppWaveShr1, 0xF>(id[u]);
                const unsigned long long heads = __ballot(lane == 0 || prev != id[u]);
                const int start = 63 - __clzll(heads & (below | (1ull << lane)));
                const T s = segmented_scan(pr[u], lane, start);
                const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
                if (tail && id[u] != (int)kPadRow) vacc[id[u]] += s;
            }
            advance(pc, cc);
        };
        do {
            step(A);
            if (pc < P) step(B);
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
    uint16_t *cnt = nullptr, *seg = nullptr;  // analysis only
    int32_t *pcs = nullptr, *sums = nullptr;
    auto release = [&]() {
        for (uint16_t *q : {cnt, seg})
            if (q) (void)hipFree(q);
        for (int32_t *q : {pcs, sums})
            if (q) (void)hipFree(q);
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
    // ranges of rows, then the virtual rows of every row (vstart[n] = all of them)
    if ((e = hipMalloc(&h->pan_range, sizeof(int32_t) * ((size_t)R + 1))) != hipSuccess ||
        (e = hipMalloc(&h->pan_vstart, sizeof(int32_t) * ((size_t)n + 1))) != hipSuccess ||
        (e = hipMalloc(&pcs, sizeof(int32_t) * (size_t)n)) != hipSuccess ||
        (e = hipMalloc(&sums, sizeof(int32_t) * (size_t)scan_sums_slots(n))) != hipSuccess)
        return fail(e, "hipMalloc(panel ranges)");
    hipLaunchKernelGGL(k_pan_ranges, dim3((R + kBlock) / kBlock), dim3(kBlock), 0, s, n, h->row_ptr, R,
                       (int64_t)h->nnz + n, h->pan_range);
    hipLaunchKernelGGL(k_pan_pieces, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, h->row_ptr, pcs);
    exclusive_scan(n, pcs, sums, h->pan_vstart, s);
    std::vector<int32_t> rr((size_t)R + 1), vs((size_t)n + 1);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(rr.data(), h->pan_range, sizeof(int32_t) * (R + 1), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(vs.data(), h->pan_vstart, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e, "panel ranges");
    for (int32_t *q : {pcs, sums}) (void)hipFree(q);
    pcs = sums = nullptr;
    for (int r = 0; r < R; ++r)
        if (vs[rr[r + 1]] - vs[rr[r]] > kPanelMaxRows) return done();  // too many for a workgroup
    const size_t V = (size_t)vs[n];
    int32_t *hp = (int32_t *)h->h_pinned;
    // entries per (virtual row, panel) -> padded segment starts and panel starts
    if ((e = hipMalloc(&cnt, sizeof(uint16_t) * V * P)) != hipSuccess ||
        (e = hipMalloc(&seg, sizeof(uint16_t) * (size_t)P * (V + R))) != hipSuccess ||
        (e = hipMalloc(&h->pan_phase, sizeof(int32_t) * (size_t)R * (P + 1))) != hipSuccess ||
        (e = hipMalloc(&h->pan_base, sizeof(int32_t) * ((size_t)R + 1))) != hipSuccess)
        return fail(e, "hipMalloc(panel layout)");
    hipLaunchKernelGGL(k_pan_zero, dim3(1), dim3(64), 0, s, h->flags);
    hipLaunchKernelGGL(k_pan_counts, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, h->row_ptr, h->col,
                       (const int32_t *)h->pan_vstart, W, P, cnt, h->flags);
    // each range's entry count (padding included, into pan_base for now) -> the
    // ranges' first entries
    hipLaunchKernelGGL(k_pan_layout, dim3(R), dim3(kPanelThreads), 0, s, P, (const int32_t *)h->pan_range,
                       (const int32_t *)h->pan_vstart, (const uint16_t *)cnt, seg, h->pan_phase,
                       h->pan_base, h->flags);
    std::vector<int32_t> tot((size_t)R);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(tot.data(), h->pan_base, sizeof(int32_t) * R, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(hp, h->flags, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e, "panel layout");
    if (hp[0] != 0) return done();  // unsorted rows or an oversized (range, panel) block
    std::vector<int32_t> rb((size_t)R + 1, 0);
    int64_t total = 0;
    for (int r = 0; r < R; ++r) {
        rb[r] = (int32_t)total;
        total += tot[r];
        if (total > INT32_MAX) return done();  // too many entries with the padding
    }
    rb[R] = (int32_t)total;
    if ((e = hipMemcpyAsync(h->pan_base, rb.data(), sizeof(int32_t) * ((size_t)R + 1), hipMemcpyHostToDevice,
                            s)) != hipSuccess ||
        (e = hipMalloc(&h->pan_val, (size_t)esz * std::max<int64_t>(total, 1))) != hipSuccess ||
        (e = hipMalloc(&h->pan_key, sizeof(uint32_t) * std::max<int64_t>(total, 1))) != hipSuccess ||
        (e = hipMalloc(&h->pan_part, (size_t)esz * kPanelGroups * n)) != hipSuccess ||
        (!h->pan_done && (e = hipEventCreateWithFlags(&h->pan_done, hipEventDisableTiming)) != hipSuccess) ||
        (e = hipMemsetAsync(h->pan_val, 0, (size_t)esz * total, s)) != hipSuccess ||
        (e = hipMemsetD32Async((hipDeviceptr_t)h->pan_key, (int)(kPadRow << 16), (size_t)total, s)) != hipSuccess)
        return fail(e, "hipMalloc(panels)");
    if (esz == 8)
        hipLaunchKernelGGL(k_pan_scatter<double>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n,
                           h->row_ptr, h->col, (const double *)h->vals, W, P, R, (const int32_t *)h->pan_range,
                           (const int32_t *)h->pan_vstart, (const uint16_t *)seg,
                           (const int32_t *)h->pan_phase, (const int32_t *)h->pan_base, (double *)h->pan_val,
                           h->pan_key);
    else
        hipLaunchKernelGGL(k_pan_scatter<float>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n,
                           h->row_ptr, h->col, (const float *)h->vals, W, P, R, (const int32_t *)h->pan_range,
                           (const int32_t *)h->pan_vstart, (const uint16_t *)seg,
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

bool use_panels(const spcg_csr *A) { return A->has_panels && panels_mode() == SPCG_PANELS_ON; }

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
    if (mode > SPCG_PANELS_ON) return SPCG_INVALID_ARG;
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
