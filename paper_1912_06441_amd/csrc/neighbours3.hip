// neighbours3.hip -- bucket-grid neighbour search in three dimensions.
//
// Neighbour set of node i (Sec. 2 of King, Lind & Nasar, with the third
// coordinate): every j != i with |r_j - r_i| < R_i, minimum image on periodic
// axes, ascending j.  The squared distance is summed x, y, z in that order
// with explicitly rounded FP64 products and sums, so the sets do not depend
// on contraction choices.  No radius growth (the critical stencil sizes the
// paper gives are two-dimensional).
#include "labfm_internal.hpp"

namespace labfm {

namespace {

__device__ inline int cell_coord3(double v, double lo, double w, int nc) {
    int c = (int)floor((v - lo) / w);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ inline double min_image3(double d, double L, int per) {
    if (!per) return d;
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

__global__ void k_bin3_count(const double* x, const double* y, const double* z, int64_t n, Grid3 g,
                             int32_t* node_cell, int32_t* cell_count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cx = cell_coord3(x[i], g.lo[0], g.w[0], g.nc[0]);
    const int cy = cell_coord3(y[i], g.lo[1], g.w[1], g.nc[1]);
    const int cz = cell_coord3(z[i], g.lo[2], g.w[2], g.nc[2]);
    const int cell = (cz * g.nc[1] + cy) * g.nc[0] + cx;
    node_cell[i] = cell;
    atomicAdd(&cell_count[cell], 1);
}

__global__ void k_bin3_scatter(int64_t n, const int32_t* node_cell, const int32_t* cell_start, int32_t* fill,
                               int32_t* idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cell = node_cell[i];
    const int pos = atomicAdd(&fill[cell], 1);
    idx[cell_start[cell] + pos] = (int32_t)i;
}

// cell range of one axis around coordinate cell c with ring r
__device__ inline void axis_range(int c, int r, int nc, int per, int& lo, int& hi) {
    if (per && 2 * r + 1 >= nc) {
        lo = 0;
        hi = nc - 1;
    } else if (per) {
        lo = c - r;
        hi = c + r;
    } else {
        lo = max(c - r, 0);
        hi = min(c + r, nc - 1);
    }
}

template <typename F>
__device__ int64_t visit3(int64_t i, double xi, double yi, double zi, double r, const double* x, const double* y,
                          const double* z, const Grid3& g, const int32_t* cell_start, const int32_t* idx, F emit) {
    const double r2 = __dmul_rn(r, r);
    const double pc[3] = {xi, yi, zi};
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int c = cell_coord3(pc[a], g.lo[a], g.w[a], g.nc[a]);
        const int ring = (int)ceil(r / g.w[a]);
        axis_range(c, ring, g.nc[a], g.per[a], lo[a], hi[a]);
    }
    int64_t cnt = 0;
    for (int zz = lo[2]; zz <= hi[2]; ++zz) {
        const int ccz = zz < 0 ? zz + g.nc[2] : (zz >= g.nc[2] ? zz - g.nc[2] : zz);
        for (int yy = lo[1]; yy <= hi[1]; ++yy) {
            const int ccy = yy < 0 ? yy + g.nc[1] : (yy >= g.nc[1] ? yy - g.nc[1] : yy);
            for (int xx = lo[0]; xx <= hi[0]; ++xx) {
                const int ccx = xx < 0 ? xx + g.nc[0] : (xx >= g.nc[0] ? xx - g.nc[0] : xx);
                const int cell = (ccz * g.nc[1] + ccy) * g.nc[0] + ccx;
                const int s1 = cell_start[cell + 1];
                for (int s = cell_start[cell]; s < s1; ++s) {
                    const int32_t j = idx[s];
                    if (j == i) continue;
                    const double dx = min_image3(__dsub_rn(x[j], xi), g.L[0], g.per[0]);
                    const double dy = min_image3(__dsub_rn(y[j], yi), g.L[1], g.per[1]);
                    const double dz = min_image3(__dsub_rn(z[j], zi), g.L[2], g.per[2]);
                    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                    if (d2 < r2) {
                        emit(cnt, j);
                        ++cnt;
                    }
                }
            }
        }
    }
    return cnt;
}

__global__ __launch_bounds__(256) void k_count3(const double* x, const double* y, const double* z, int64_t n,
                                                Grid3 g, const int32_t* cell_start, const int32_t* idx,
                                                const double* R, int64_t* counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    auto none = [](int64_t, int32_t) {};
    counts[i] = visit3(i, x[i], y[i], z[i], R[i], x, y, z, g, cell_start, idx, none);
}

__global__ __launch_bounds__(256) void k_fill3(const double* x, const double* y, const double* z, int64_t n,
                                               Grid3 g, const int32_t* cell_start, const int32_t* idx,
                                               const double* R, const int64_t* row_ptr, int32_t* col) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t* out = col + row_ptr[i];
    const int64_t cap = row_ptr[i + 1] - row_ptr[i];
    visit3(i, x[i], y[i], z[i], R[i], x, y, z, g, cell_start, idx, [&](int64_t c, int32_t j) {
        if (c < cap) out[c] = j;
    });
}

labfm_err build_grid3(Context* c, const double* x, const double* y, const double* z, int64_t n, const Grid3& g,
                      hipStream_t st) {
    const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    labfm_err e;
    if ((e = ensure(c->grid_count, sizeof(int32_t) * (size_t)(2 * ncell + 1))) != LABFM_OK) return e;
    if ((e = ensure(c->grid_idx, sizeof(int32_t) * (size_t)(n + 1))) != LABFM_OK) return e;
    if ((e = ensure(c->node_cell, sizeof(int32_t) * (size_t)(n + 1))) != LABFM_OK) return e;
    int32_t* count = (int32_t*)c->grid_count.p;  // [ncell] counters, reused as fill pointers
    int32_t* start = count + ncell;               // [ncell + 1]
    LABFM_HIP_CHECK(hipMemsetAsync(count, 0, sizeof(int32_t) * (size_t)ncell, st));
    const unsigned nb = (unsigned)((n + 255) / 256);
    k_bin3_count<<<nb, 256, 0, st>>>(x, y, z, n, g, (int32_t*)c->node_cell.p, count);
    if ((e = exclusive_scan_i32(c, count, start, ncell, st)) != LABFM_OK) return e;
    LABFM_HIP_CHECK(hipMemsetAsync(count, 0, sizeof(int32_t) * (size_t)ncell, st));
    k_bin3_scatter<<<nb, 256, 0, st>>>(n, (const int32_t*)c->node_cell.p, start, count, (int32_t*)c->grid_idx.p);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

}  // namespace

labfm_err neighbours3_count(Context* c, const double* x, const double* y, const double* z, int64_t n,
                            const Grid3& g, const double* R, int64_t* row_ptr, hipStream_t st) {
    labfm_err e = build_grid3(c, x, y, z, n, g, st);
    if (e != LABFM_OK) return e;
    if ((e = ensure(c->counts, sizeof(int64_t) * (size_t)(n + 1))) != LABFM_OK) return e;
    int64_t* counts = (int64_t*)c->counts.p;
    const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    const int32_t* start = (const int32_t*)c->grid_count.p + ncell;
    KernelTimer timer(c, "neigh3_count", st);
    k_count3<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(x, y, z, n, g, start, (const int32_t*)c->grid_idx.p, R,
                                                          counts);
    LABFM_HIP_CHECK(hipGetLastError());
    return exclusive_scan_i64(c, counts, row_ptr, n, st);
}

labfm_err neighbours3_fill(Context* c, const double* x, const double* y, const double* z, int64_t n,
                           const Grid3& g, const double* R, const int64_t* row_ptr, int32_t* col, hipStream_t st) {
    labfm_err e = build_grid3(c, x, y, z, n, g, st);
    if (e != LABFM_OK) return e;
    const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    const int32_t* start = (const int32_t*)c->grid_count.p + ncell;
    KernelTimer timer(c, "neigh3_fill", st);
    k_fill3<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(x, y, z, n, g, start, (const int32_t*)c->grid_idx.p, R,
                                                         row_ptr, col);
    LABFM_HIP_CHECK(hipGetLastError());
    return sort_rows(row_ptr, col, n, st);
}

}  // namespace labfm
