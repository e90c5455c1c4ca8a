// Error state, device allocation, workspace and a device exclusive scan.
#include "internal.hpp"

#include <cstring>

namespace dgo {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

dgo_status hip_fail(hipError_t e, const char *what, const char *file, int line) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    set_error(buf);
    (void)hipGetLastError();  // clear the sticky-free error slot
    return e == hipErrorOutOfMemory ? DGO_ERR_NOMEM : DGO_ERR_DEVICE;
}

void *Alloc::get(size_t bytes, hipStream_t s) const {
    if (bytes == 0) bytes = 256;
    if (has_user) return user.alloc(bytes, (dgo_stream)s, user.ctx);
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void Alloc::put(void *p, hipStream_t s) const {
    if (!p) return;
    if (has_user) {
        user.free(p, (dgo_stream)s, user.ctx);
        return;
    }
    (void)hipFreeAsync(p, s);
}

dgo_status mesh_workspace(dgo_mesh *m, size_t bytes, hipStream_t s, void **out) {
    if (bytes > m->ws_bytes) {
        m->alloc.put(m->ws, s);
        m->ws = nullptr;
        m->ws_bytes = 0;
        size_t want = bytes + bytes / 4;
        void *p = m->alloc.get(want, s);
        if (!p) return fail(DGO_ERR_NOMEM, "workspace allocation failed");
        m->ws = p;
        m->ws_bytes = want;
    }
    *out = m->ws;
    return DGO_OK;
}


// ------------------------------------------------------------------ scan

constexpr int SCAN_T = 256;
constexpr int SCAN_IPT = 4;
constexpr int SCAN_TILE = SCAN_T * SCAN_IPT;

// Each workgroup scans SCAN_TILE consecutive values (exclusive) and stores
// the tile total in sums[blockIdx.x]. Every thread writes only the entries it
// read, so in == out is allowed.
__global__ void __launch_bounds__(SCAN_T)
k_scan_tile(const int32_t *in, int32_t *out, int64_t n, int32_t *sums) {
    __shared__ int32_t sh[SCAN_T];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_IPT;
    int32_t v[SCAN_IPT];
    int32_t acc = 0;
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        acc += v[i];
    }
    sh[t] = acc;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int32_t add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int32_t run = sh[t] - acc;
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (t == SCAN_T - 1) sums[blockIdx.x] = sh[t];
}

__global__ void k_scan_add(int32_t *out, int64_t n, const int32_t *sums, int64_t nb) {
    const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    const int32_t off = sums[blockIdx.x];
#pragma unroll
    for (int r = 0; r < SCAN_IPT; ++r) {
        int64_t j = i + (int64_t)r * SCAN_T;
        if (j < n) out[j] += off;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

__global__ void k_set_zero_total(int32_t *out) { out[0] = 0; }

size_t scan_tmp_elems(int64_t n) {
    if (n <= SCAN_TILE) return 0;
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    return (size_t)(nb + 1) + scan_tmp_elems(nb);
}

dgo_status exclusive_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp,
                          hipStream_t s) {
    if (n <= 0) {
        k_set_zero_total<<<1, 1, 0, s>>>(out);
        DGO_HIP(hipGetLastError());
        return DGO_OK;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        k_scan_tile<<<1, SCAN_T, 0, s>>>(in, out, n, out + n);
        DGO_HIP(hipGetLastError());
        return DGO_OK;
    }
    int32_t *sums = tmp;
    k_scan_tile<<<(unsigned)nb, SCAN_T, 0, s>>>(in, out, n, sums);
    DGO_HIP(hipGetLastError());
    DGO_TRY(exclusive_scan(sums, sums, nb, tmp + nb + 1, s));
    k_scan_add<<<(unsigned)nb, SCAN_T, 0, s>>>(out, n, sums, nb);
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}

}  // namespace dgo

extern "C" const char *dgo_last_error(void) { return dgo::g_last_error.c_str(); }

extern "C" const char *dgo_version(void) { return "dgo 0.1 gfx950"; }
