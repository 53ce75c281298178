// neighbours.hip -- bucket-grid neighbour search on gfx950 and device-wide scans.
//
// Neighbour set of node i (Sec. 2 of King, Lind & Nasar): every j != i with
// |r_j - r_i| < R_i (R_i = 2 h_i), minimum image on periodic axes, ascending j.
// Optional count-driven radius growth to the critical stencil sizes of
// Sec. 3.2.  The distance test is evaluated with explicitly rounded FP64
// products and sums so that it is identical on any IEEE FP64 host.
#include "labfm_internal.hpp"

namespace labfm {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__device__ T block_exclusive_scan(T v, T* lds, T& total) {
    // Hillis-Steele inclusive scan over SCAN_THREADS values in LDS
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        T add = (t >= off) ? lds[t - off] : T(0);
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    total = lds[SCAN_THREADS - 1];
    T incl = lds[t];
    __syncthreads();
    return incl - v;
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const T* in, T* out, T* tile_sums, int64_t n) {
    __shared__ T lds[SCAN_THREADS];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        v[q] = (base + q < n) ? in[base + q] : T(0);
        s += v[q];
    }
    T total;
    T run = block_exclusive_scan<T>(s, lds, total);
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// single block: exclusive scan of the tile sums in chunks, carrying the total
template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(T* sums, int64_t ntiles, T* out_total) {
    __shared__ T lds[SCAN_THREADS];
    T carry = 0;
    for (int64_t c0 = 0; c0 < ntiles; c0 += SCAN_TILE) {
        int64_t base = c0 + (int64_t)threadIdx.x * SCAN_ITEMS;
        T v[SCAN_ITEMS];
        T s = 0;
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS; ++q) {
            v[q] = (base + q < ntiles) ? sums[base + q] : T(0);
            s += v[q];
        }
        T total;
        T run = block_exclusive_scan<T>(s, lds, total) + carry;
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS; ++q) {
            if (base + q < ntiles) sums[base + q] = run;
            run += v[q];
        }
        carry += total;
    }
    if (threadIdx.x == 0) *out_total = carry;
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(T* out, const T* tile_offsets, int64_t n) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T off = tile_offsets[blockIdx.x];
    for (int q = threadIdx.x; q < SCAN_TILE; q += SCAN_THREADS) {
        int64_t i = base + q;
        if (i < n) out[i] += off;
    }
}

template <typename T>
labfm_err scan_impl(Context* c, const T* in, T* out, int64_t n, hipStream_t st) {
    // out has n+1 entries; out[n] = total
    int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles == 0) {
        LABFM_HIP_CHECK(hipMemsetAsync(out, 0, sizeof(T), st));
        return LABFM_OK;
    }
    labfm_err e = ensure(c->scan_tmp, sizeof(T) * (size_t)ntiles);
    if (e != LABFM_OK) return e;
    T* sums = (T*)c->scan_tmp.p;
    k_scan_tiles<T><<<(unsigned)ntiles, SCAN_THREADS, 0, st>>>(in, out, sums, n);
    k_scan_sums<T><<<1, SCAN_THREADS, 0, st>>>(sums, ntiles, out + n);
    k_scan_add<T><<<(unsigned)ntiles, SCAN_THREADS, 0, st>>>(out, sums, n);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

// ---------------------------------------------------------------------------
// bucket grid

__device__ inline int cell_coord(double v, double lo, double w, int nc) {
    int c = (int)floor((v - lo) / w);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_bin_count(const double* x, const double* y, int64_t n, GridSpec g, int32_t* node_cell,
                            int32_t* cell_count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(x[i], g.lox, g.wx, g.ncx);
    int cy = cell_coord(y[i], g.loy, g.wy, g.ncy);
    int cell = cy * g.ncx + cx;
    node_cell[i] = cell;
    atomicAdd(&cell_count[cell], 1);
}

__global__ void k_bin_scatter(int64_t n, const int32_t* node_cell, const int32_t* cell_start,
                              int32_t* fill, int32_t* idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cell = node_cell[i];
    int pos = atomicAdd(&fill[cell], 1);
    idx[cell_start[cell] + pos] = (int32_t)i;
}

__device__ inline double min_image(double d, double L, int per) {
    if (!per) return d;
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

__device__ inline int ncrit_of(int k) { return k <= 2 ? 8 : (k <= 4 ? 21 : (k <= 6 ? 37 : 57)); }

// Visit every j within radius r of node i; `emit(j)` is called for each.
template <typename F>
__device__ int64_t visit(int64_t i, double xi, double yi, double r, const double* x, const double* y,
                         const GridSpec& g, const int32_t* cell_start, const int32_t* idx, F emit) {
    const double r2 = __dmul_rn(r, r);
    int cx = cell_coord(xi, g.lox, g.wx, g.ncx);
    int cy = cell_coord(yi, g.loy, g.wy, g.ncy);
    int rx = (int)ceil(r / g.wx), ry = (int)ceil(r / g.wy);
    int x0, x1, y0, y1;
    if (g.perx && 2 * rx + 1 >= g.ncx) { x0 = 0; x1 = g.ncx - 1; }
    else if (g.perx) { x0 = cx - rx; x1 = cx + rx; }
    else { x0 = max(cx - rx, 0); x1 = min(cx + rx, g.ncx - 1); }
    if (g.pery && 2 * ry + 1 >= g.ncy) { y0 = 0; y1 = g.ncy - 1; }
    else if (g.pery) { y0 = cy - ry; y1 = cy + ry; }
    else { y0 = max(cy - ry, 0); y1 = min(cy + ry, g.ncy - 1); }
    int64_t cnt = 0;
    for (int yy = y0; yy <= y1; ++yy) {
        int ccy = yy < 0 ? yy + g.ncy : (yy >= g.ncy ? yy - g.ncy : yy);
        for (int xx = x0; xx <= x1; ++xx) {
            int ccx = xx < 0 ? xx + g.ncx : (xx >= g.ncx ? xx - g.ncx : xx);
            int cell = ccy * g.ncx + ccx;
            int s1 = cell_start[cell + 1];
            for (int s = cell_start[cell]; s < s1; ++s) {
                int32_t j = idx[s];
                if (j == i) continue;
                double dx = min_image(__dsub_rn(x[j], xi), g.Lx, g.perx);
                double dy = min_image(__dsub_rn(y[j], yi), g.Ly, g.pery);
                double d2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
                if (d2 < r2) {
                    emit(cnt, j);
                    ++cnt;
                }
            }
        }
    }
    return cnt;
}

__global__ __launch_bounds__(256) void k_count(const double* x, const double* y, int64_t n, GridSpec g,
                                               const int32_t* cell_start, const int32_t* idx, double* R,
                                               const int8_t* order, int grow, int max_grow, int64_t* counts) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double xi = x[i], yi = y[i], r = R[i];
    auto none = [](int64_t, int32_t) {};
    int64_t c = visit(i, xi, yi, r, x, y, g, cell_start, idx, none);
    if (grow) {
        int need = ncrit_of(order[i]);
        int it = 0;
        while (c < need && it < max_grow) {
            r = __dmul_rn(r, 1.1);
            c = visit(i, xi, yi, r, x, y, g, cell_start, idx, none);
            ++it;
        }
        R[i] = r;
    }
    counts[i] = c;
}

__global__ __launch_bounds__(256) void k_fill(const double* x, const double* y, int64_t n, GridSpec g,
                                              const int32_t* cell_start, const int32_t* idx, const double* R,
                                              const int64_t* row_ptr, int32_t* col) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t* out = col + row_ptr[i];
    int64_t cap = row_ptr[i + 1] - row_ptr[i];
    visit(i, x[i], y[i], R[i], x, y, g, cell_start, idx, [&](int64_t c, int32_t j) {
        if (c < cap) out[c] = j;
    });
}

// One wave per row: rank sort (row entries are distinct).
constexpr int SORT_WAVES = 4;
constexpr int SORT_CAP = 512;
__global__ __launch_bounds__(64 * SORT_WAVES) void k_sort_rows(const int64_t* row_ptr, int32_t* col, int64_t n) {
    __shared__ int32_t buf[SORT_WAVES][SORT_CAP];
    int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    int64_t row = (int64_t)blockIdx.x * SORT_WAVES + w;
    int64_t s = 0, len = 0;
    if (row < n) {
        s = row_ptr[row];
        len = row_ptr[row + 1] - s;
    }
    bool in_lds = len <= SORT_CAP;
    if (in_lds)
        for (int64_t q = lane; q < len; q += 64) buf[w][q] = col[s + q];
    __syncthreads();
    if (in_lds) {
        for (int64_t q = lane; q < len; q += 64) {
            int32_t v = buf[w][q];
            int rank = 0;
            for (int64_t t = 0; t < len; ++t) rank += buf[w][t] < v;
            col[s + rank] = v;
        }
    } else if (lane == 0) {
        for (int64_t a = 1; a < len; ++a) {  // long rows: insertion sort in place
            int32_t v = col[s + a];
            int64_t b = a - 1;
            while (b >= 0 && col[s + b] > v) {
                col[s + b + 1] = col[s + b];
                --b;
            }
            col[s + b + 1] = v;
        }
    }
}

labfm_err build_grid(Context* c, const double* x, const double* y, int64_t n, const GridSpec& g,
                     hipStream_t st) {
    int64_t ncell = (int64_t)g.ncx * g.ncy;
    labfm_err e;
    if ((e = ensure(c->grid_count, sizeof(int32_t) * (size_t)(2 * ncell + 1))) != LABFM_OK) return e;
    if ((e = ensure(c->grid_idx, sizeof(int32_t) * (size_t)(n + 1))) != LABFM_OK) return e;
    if ((e = ensure(c->node_cell, sizeof(int32_t) * (size_t)(n + 1))) != LABFM_OK) return e;
    int32_t* count = (int32_t*)c->grid_count.p;     // [ncell] counters, reused as fill pointers
    int32_t* start = count + ncell;                  // [ncell + 1]
    LABFM_HIP_CHECK(hipMemsetAsync(count, 0, sizeof(int32_t) * (size_t)ncell, st));
    unsigned nb = (unsigned)((n + 255) / 256);
    k_bin_count<<<nb, 256, 0, st>>>(x, y, n, g, (int32_t*)c->node_cell.p, count);
    if ((e = scan_impl<int32_t>(c, count, start, ncell, st)) != LABFM_OK) return e;
    LABFM_HIP_CHECK(hipMemsetAsync(count, 0, sizeof(int32_t) * (size_t)ncell, st));
    k_bin_scatter<<<nb, 256, 0, st>>>(n, (const int32_t*)c->node_cell.p, start, count, (int32_t*)c->grid_idx.p);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

}  // namespace

labfm_err exclusive_scan_i64(Context* c, const int64_t* in, int64_t* out, int64_t n, hipStream_t st) {
    return scan_impl<int64_t>(c, in, out, n, st);
}
labfm_err exclusive_scan_i32(Context* c, const int32_t* in, int32_t* out, int64_t n, hipStream_t st) {
    return scan_impl<int32_t>(c, in, out, n, st);
}

labfm_err sort_rows(const int64_t* row_ptr, int32_t* col, int64_t n, hipStream_t st) {
    if (n <= 0) return LABFM_OK;
    unsigned ns = (unsigned)((n + SORT_WAVES - 1) / SORT_WAVES);
    k_sort_rows<<<ns, 64 * SORT_WAVES, 0, st>>>(row_ptr, col, n);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err neighbours_count(Context* c, const double* x, const double* y, int64_t n, const GridSpec& g,
                           double* R, const int8_t* order, int grow, int max_grow, int64_t* row_ptr,
                           hipStream_t st) {
    labfm_err e = build_grid(c, x, y, n, g, st);
    if (e != LABFM_OK) return e;
    if ((e = ensure(c->counts, sizeof(int64_t) * (size_t)(n + 1))) != LABFM_OK) return e;
    int64_t* counts = (int64_t*)c->counts.p;
    int64_t ncell = (int64_t)g.ncx * g.ncy;
    const int32_t* start = (const int32_t*)c->grid_count.p + ncell;
    unsigned nb = (unsigned)((n + 255) / 256);
    KernelTimer timer(c, "neigh_count", st);
    k_count<<<nb, 256, 0, st>>>(x, y, n, g, start, (const int32_t*)c->grid_idx.p, R, order, grow, max_grow,
                                counts);
    LABFM_HIP_CHECK(hipGetLastError());
    return exclusive_scan_i64(c, counts, row_ptr, n, st);
}

labfm_err neighbours_fill(Context* c, const double* x, const double* y, int64_t n, const GridSpec& g,
                          const double* R, const int64_t* row_ptr, int32_t* col, hipStream_t st) {
    labfm_err e = build_grid(c, x, y, n, g, st);
    if (e != LABFM_OK) return e;
    int64_t ncell = (int64_t)g.ncx * g.ncy;
    const int32_t* start = (const int32_t*)c->grid_count.p + ncell;
    unsigned nb = (unsigned)((n + 255) / 256);
    KernelTimer timer(c, "neigh_fill", st);
    k_fill<<<nb, 256, 0, st>>>(x, y, n, g, start, (const int32_t*)c->grid_idx.p, R, row_ptr, col);
    unsigned ns = (unsigned)((n + SORT_WAVES - 1) / SORT_WAVES);
    k_sort_rows<<<ns, 64 * SORT_WAVES, 0, st>>>(row_ptr, col, n);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

}  // namespace labfm
