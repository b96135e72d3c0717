// Graph upload, validation and the exact device edge hash.
//
// The paper tests edge membership with a lossy byte map indexed by a 32-bit hash of the
// vertex pair, where collisions read as edges (Sec. III-C).  This library needs exact
// membership, so the hash here is an open-addressing table of the m undirected edges
// with full 64-bit keys (min << 32 | max), linear probing, capacity the power of two
// >= 2m (load factor <= 0.5).  It is the authority for CSR validation (symmetry),
// gempe_has_edge, and the edge-hit count of every loss evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.h"

namespace {

constexpr int kBlock = 256;

// status bits and the two entry counters live in g->status_dev:
//   [0] status bits, [1] unused, [2..3] int64 count of entries with i<j, [4..5] i>j.
__global__ void k_check_row_ptr(const int64_t *__restrict__ row_ptr, int n, int64_t nnz,
                                unsigned *status) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t v = row_ptr[i];
    bool bad = v < 0 || v > nnz;
    if (i == 0) bad |= v != 0;
    if (i == n) bad |= v != nnz;
    if (i < n) bad |= row_ptr[i + 1] < v;
    if (bad) atomicOr(status, kStatusBadRowPtr);
}

// Row of CSR entry e by binary search over row_ptr (valid once row_ptr is monotone).
__global__ void k_coo_rows(const int64_t *__restrict__ row_ptr, int n, int64_t nnz,
                           int32_t *__restrict__ coo_row) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int lo = 0, hi = n - 1;  // largest i with row_ptr[i] <= e
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    coo_row[e] = lo;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, uint64_t count) {
    uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = v;
}

// Per entry: range, self-loop and ordering checks; entries with i < j insert their key.
__global__ void k_check_insert(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                               const int32_t *__restrict__ coo_row, int n, int64_t nnz,
                               unsigned long long *__restrict__ table, unsigned long long cap,
                               unsigned *status, unsigned long long *upper_count) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int i = coo_row[e];
    int j = col[e];
    if (j < 0 || j >= n || j == i) {
        atomicOr(status, kStatusBadCol);
        return;
    }
    if (e + 1 < row_ptr[i + 1] && col[e + 1] <= j) atomicOr(status, kStatusUnsorted);
    if (i < j) {
        atomicAdd(upper_count, 1ull);
        unsigned long long key = gempe_edge_key(i, j), mask = cap - 1;
        unsigned long long s = gempe_mix64(key) & mask;
        for (unsigned long long probe = 0;; ++probe) {
            if (probe >= cap) {
                atomicOr(status, kStatusHashFull);
                return;
            }
            unsigned long long prev = atomicCAS(&table[s], kHashEmpty, key);
            if (prev == kHashEmpty) return;
            if (prev == key) {  // the same undirected edge twice in row i
                atomicOr(status, kStatusUnsorted);
                return;
            }
            s = (s + 1) & mask;
        }
    }
}

// Entries with i > j must find their mirror (j, i) in the table.
__global__ void k_check_mirror(const int32_t *__restrict__ col, const int32_t *__restrict__ coo_row,
                               int64_t nnz, const unsigned long long *__restrict__ table,
                               unsigned long long cap, unsigned *status,
                               unsigned long long *lower_count) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int i = coo_row[e];
    int j = col[e];
    if (i > j) {
        atomicAdd(lower_count, 1ull);
        if (!gempe_hash_contains(table, cap, gempe_edge_key(i, j)))
            atomicOr(status, kStatusAsymmetric);
    }
}

__global__ void k_has_edge(const unsigned long long *__restrict__ table, unsigned long long cap,
                           int n, int64_t q, const int32_t *__restrict__ qi,
                           const int32_t *__restrict__ qj, uint8_t *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= q) return;
    int a = qi[k], b = qj[k];
    bool ok = a >= 0 && a < n && b >= 0 && b < n && a != b;
    out[k] = (ok && cap > 0 && gempe_hash_contains(table, cap, gempe_edge_key(a, b))) ? 1 : 0;
}

unsigned blocks_for(int64_t count) {
    return (unsigned)std::max<int64_t>(1, (count + kBlock - 1) / kBlock);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct GraphOffsets {
    size_t row_ptr, col_idx, coo_row, hash, status, total;
};

GraphOffsets graph_offsets(int32_t n, int64_t nnz, uint64_t cap) {
    GraphOffsets o;
    size_t off = 0;
    o.status = off;
    off += 256;
    o.row_ptr = off;
    off = align256(off + sizeof(int64_t) * ((size_t)n + 1));
    o.col_idx = off;
    off = align256(off + sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
    o.coo_row = off;
    off = align256(off + sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
    o.hash = off;
    off = align256(off + sizeof(unsigned long long) * cap);
    o.total = off;
    return o;
}

uint64_t hash_capacity(int64_t m) {
    uint64_t cap = 2;
    while (cap < 2 * (uint64_t)m) cap <<= 1;
    return cap;
}

}  // namespace

gempe_status gempe_graph_check_args(int32_t n, int64_t nnz, const void *row_ptr, const void *col_idx,
                                    const char *who) {
    const std::string w(who);
    if (n < 1) return gempe_fail(GEMPE_ERR_ARG, w + ": n must be >= 1");
    if (nnz < 0 || (nnz & 1)) return gempe_fail(GEMPE_ERR_GRAPH, w + ": nnz must be even and >= 0");
    if ((uint64_t)nnz > (uint64_t)n * (uint64_t)(n - 1))
        return gempe_fail(GEMPE_ERR_GRAPH, w + ": nnz exceeds n(n-1)");
    if (!row_ptr || (nnz > 0 && !col_idx)) return gempe_fail(GEMPE_ERR_ARG, w + ": null CSR pointer");
    return GEMPE_OK;
}

size_t gempe_graph_mem_bytes(int32_t n, int64_t nnz) {
    return graph_offsets(n, nnz, hash_capacity(nnz / 2)).total;
}

gempe_status gempe_graph_build(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                               hipMemcpyKind kind, void *mem, hipStream_t stream, gempe_graph_s *g) {
    g->n = n;
    g->nnz = nnz;
    g->m = nnz / 2;
    GEMPE_HIP_TRY(hipGetDevice(&g->device));
    const uint64_t cap = hash_capacity(g->m);
    g->hash_cap = cap;
    const GraphOffsets o = graph_offsets(n, nnz, cap);
    unsigned char *base = static_cast<unsigned char *>(mem);
    g->mem = mem;
    g->status_dev = reinterpret_cast<unsigned *>(base + o.status);
    g->row_ptr = reinterpret_cast<int64_t *>(base + o.row_ptr);
    g->col_idx = reinterpret_cast<int32_t *>(base + o.col_idx);
    g->coo_row = reinterpret_cast<int32_t *>(base + o.coo_row);
    g->hash = reinterpret_cast<unsigned long long *>(base + o.hash);

    GEMPE_HIP_TRY(hipMemsetAsync(g->status_dev, 0, 256, stream));
    GEMPE_HIP_TRY(hipMemcpyAsync(g->row_ptr, row_ptr, sizeof(int64_t) * (n + 1), kind, stream));
    if (nnz > 0) GEMPE_HIP_TRY(hipMemcpyAsync(g->col_idx, col_idx, sizeof(int32_t) * nnz, kind, stream));
    unsigned *status = g->status_dev;
    unsigned long long *upper = reinterpret_cast<unsigned long long *>(g->status_dev + 2);
    unsigned long long *lower = reinterpret_cast<unsigned long long *>(g->status_dev + 4);

    // 1. row_ptr shape; everything after indexes through it, so stop here if it is bad.
    k_check_row_ptr<<<blocks_for(n + 1), kBlock, 0, stream>>>(g->row_ptr, n, nnz, status);
    GEMPE_HIP_TRY(hipGetLastError());
    unsigned host_status = 0;
    GEMPE_HIP_TRY(hipMemcpyAsync(&host_status, status, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
    GEMPE_HIP_TRY(hipStreamSynchronize(stream));
    if (host_status) return gempe_fail(GEMPE_ERR_GRAPH, "graph_create: row_ptr is not a valid CSR offset array");
    // 2. entry checks, hash insertion of the i<j half, mirror lookups of the i>j half.
    k_fill_u64<<<blocks_for((int64_t)cap), kBlock, 0, stream>>>(g->hash, kHashEmpty, cap);
    if (nnz > 0) {
        k_coo_rows<<<blocks_for(nnz), kBlock, 0, stream>>>(g->row_ptr, n, nnz, g->coo_row);
        k_check_insert<<<blocks_for(nnz), kBlock, 0, stream>>>(g->row_ptr, g->col_idx, g->coo_row, n, nnz,
                                                                g->hash, cap, status, upper);
        k_check_mirror<<<blocks_for(nnz), kBlock, 0, stream>>>(g->col_idx, g->coo_row, nnz, g->hash, cap,
                                                                status, lower);
    }
    GEMPE_HIP_TRY(hipGetLastError());
    unsigned host_words[6] = {0, 0, 0, 0, 0, 0};
    GEMPE_HIP_TRY(hipMemcpyAsync(host_words, status, sizeof(host_words), hipMemcpyDeviceToHost, stream));
    GEMPE_HIP_TRY(hipStreamSynchronize(stream));
    unsigned long long nup, nlo;
    std::memcpy(&nup, host_words + 2, 8);
    std::memcpy(&nlo, host_words + 4, 8);
    unsigned bits = host_words[0];
    if (bits || nup != nlo || (int64_t)(nup + nlo) != nnz) {
        std::string why;
        if (bits & kStatusBadCol) why += " column id out of range or self-loop;";
        if (bits & kStatusUnsorted) why += " row not strictly ascending (duplicate or unsorted);";
        if (bits & kStatusAsymmetric) why += " (i,j) without (j,i);";
        if (bits & kStatusHashFull) why += " edge hash full;";
        if (!bits) why += " directed entry counts i<j and i>j differ;";
        return gempe_fail(GEMPE_ERR_GRAPH, "graph_create:" + why);
    }
    return GEMPE_OK;
}

extern "C" size_t gempe_graph_workspace_bytes(int32_t n, int64_t nnz) {
    if (gempe_graph_check_args(n, nnz, "", "", "graph_workspace_bytes") != GEMPE_OK) return 0;
    return gempe_graph_mem_bytes(n, nnz);
}

extern "C" gempe_status gempe_graph_create(int32_t n, int64_t nnz, const int64_t *row_ptr,
                                           const int32_t *col_idx, void *ws, size_t ws_bytes,
                                           hipStream_t stream, gempe_graph *out) {
    if (!out) return gempe_fail(GEMPE_ERR_ARG, "graph_create: out is NULL");
    *out = nullptr;
    gempe_status st = gempe_graph_check_args(n, nnz, row_ptr, col_idx, "graph_create");
    if (st != GEMPE_OK) return st;
    if (!ws) return gempe_fail(GEMPE_ERR_ARG, "graph_create: null workspace");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return gempe_fail(GEMPE_ERR_ARG, "graph_create: workspace must be 256-byte aligned");
    const size_t need = gempe_graph_mem_bytes(n, nnz);
    if (ws_bytes < need)
        return gempe_fail(GEMPE_ERR_NOMEM, "graph_create: workspace of " + std::to_string(ws_bytes) +
                                               " bytes, need " + std::to_string(need));
    gempe_graph_s *g = new gempe_graph_s();
    st = gempe_graph_build(n, nnz, row_ptr, col_idx, hipMemcpyDeviceToDevice, ws, stream, g);
    if (st != GEMPE_OK) {
        // nothing may still be running on the caller's memory when the error returns
        (void)hipStreamSynchronize(stream);
        delete g;
        return st;
    }
    *out = g;
    return GEMPE_OK;
}

extern "C" gempe_status gempe_graph_destroy(gempe_graph g) {
    if (!g) return gempe_fail(GEMPE_ERR_ARG, "graph_destroy: null handle");
    if (g->server_owned) return gempe_fail(GEMPE_ERR_ARG, "graph_destroy: handle is owned by a server");
    // the device memory belongs to the caller; only the host-side handle is released
    delete g;
    return GEMPE_OK;
}

extern "C" int32_t gempe_graph_num_vertices(gempe_graph g) { return g ? g->n : -1; }
extern "C" int64_t gempe_graph_num_edges(gempe_graph g) { return g ? g->m : -1; }

extern "C" gempe_status gempe_has_edge(gempe_graph g, int64_t q, const int32_t *qi, const int32_t *qj,
                                       uint8_t *out, hipStream_t stream) {
    if (!g) return gempe_fail(GEMPE_ERR_ARG, "has_edge: null handle");
    if (q < 0) return gempe_fail(GEMPE_ERR_ARG, "has_edge: q < 0");
    if (q == 0) return GEMPE_OK;
    if (!qi || !qj || !out) return gempe_fail(GEMPE_ERR_ARG, "has_edge: null pointer");
    k_has_edge<<<blocks_for(q), kBlock, 0, stream>>>(g->hash, g->hash_cap, g->n, q, qi, qj, out);
    GEMPE_HIP_TRY(hipGetLastError());
    return GEMPE_OK;
}
