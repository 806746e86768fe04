// pattern.hip -- CSR pattern of the global tangent from the connectivity
// (App. E, Alg. E1: the pattern is fixed for a mesh, so it is built once and
// the element matrices are later scattered straight into its value array).
//
// Steps, all on the device:
//   1. node -> element incidence by counting and a prefix scan;
//   2. per node, the sorted unique list of nodes sharing an element (<= 64):
//      one wave per node sorts the (element, node) candidates of up to 8
//      incident elements across its lanes and keeps the first of equal ones;
//   3. row_ptr from a scan of the neighbour counts (rows of one node have
//      equal length 3*deg);
//   4. col_idx rows and elem_rank (position of node J in node I's list),
//      written by the same wave per node.
#include <hip/hip_runtime.h>

#include "fem_internal.h"

namespace fem {
namespace {

constexpr int kMaxNbr = 64;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

enum { ERR_RANGE = 1, ERR_ORPHAN = 2, ERR_DEGREE = 4 };

__global__ void count_incidence(const int32_t* __restrict__ conn, int64_t n_entries, int32_t n_nodes,
                                int32_t* __restrict__ cnt, int32_t* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_entries) return;
    const int32_t n = conn[i];
    if (n < 0 || n >= n_nodes) {
        atomicOr(err, ERR_RANGE);
        return;
    }
    atomicAdd(&cnt[n], 1);
}

__global__ void fill_incidence(const int32_t* __restrict__ conn, int64_t n_entries, int32_t n_nodes,
                               const int64_t* __restrict__ inc_ptr, int32_t* __restrict__ fillc,
                               int32_t* __restrict__ inc) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_entries) return;
    const int32_t n = conn[i];
    if (n < 0 || n >= n_nodes) return;
    const int32_t pos = atomicAdd(&fillc[n], 1);
    inc[inc_ptr[n] + pos] = (int32_t)i;  // conn entry 8e + local index
}

// Sorted unique neighbour list of node n (n included).  Returns the count or
// -1 if it exceeds kMaxNbr.
__device__ int node_neighbours(int32_t n, const int32_t* __restrict__ conn, const int64_t* __restrict__ inc_ptr,
                               const int32_t* __restrict__ inc, int32_t* nb) {
    int cnt = 0;
    for (int64_t k = inc_ptr[n]; k < inc_ptr[n + 1]; ++k) {
        const int64_t e = inc[k] >> 3;
        for (int j = 0; j < 8; ++j) {
            const int32_t v = conn[e * 8 + j];
            // insertion into the sorted list
            int pos = cnt;
            while (pos > 0 && nb[pos - 1] > v) --pos;
            if (pos > 0 && nb[pos - 1] == v) continue;
            if (cnt == kMaxNbr) return -1;
            for (int t = cnt; t > pos; --t) nb[t] = nb[t - 1];
            nb[pos] = v;
            ++cnt;
        }
    }
    return cnt;
}

// ---- one wave per node (nodes with at most 8 incident elements; a node with
// more takes the serial node_neighbours in lane 0)

constexpr int kPatWaves = 4;  // nodes (waves) per workgroup

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ascending bitonic sort of one 64-bit key per lane across the wave.
__device__ inline uint64_t wave_sort64(uint64_t key, int lane) {
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint64_t other = __shfl_xor(key, j, 64);
            const bool keep_min = (((lane & j) == 0) == ((lane & k) == 0));
            key = keep_min ? (other < key ? other : key) : (other > key ? other : key);
        }
    return key;
}

// Lane (k, j) proposes node j of incident element k (k < 8); after the sort,
// the sorted position p knows whether it starts a new value and that value's
// index among the unique ones.  Returns the number of unique neighbours.
struct WaveNbr {
    int deg;
    bool first;     // sorted position p holds the first copy of its value
    int32_t value;  // value at sorted position p
    int uidx;       // its index among the unique values
    int origin;     // lane whose candidate sits at position p (-1: none)
};
__device__ inline WaveNbr wave_neighbours(uint64_t key, int lane) {
    key = wave_sort64(key, lane);
    const bool valid = key != ~0ull;
    const uint64_t prev = __shfl_up(key, 1, 64);
    const bool first = valid && (lane == 0 || (prev >> 32) != (key >> 32));
    const uint64_t mask = __ballot(first);
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    WaveNbr r;
    r.deg = __popcll(mask);
    r.first = first;
    r.value = (int32_t)(key >> 32);
    r.uidx = __popcll(mask & upto) - 1;
    r.origin = valid ? (int)(key & 63) : -1;
    return r;
}

__global__ __launch_bounds__(64 * kPatWaves) void node_degree_w(int32_t n_nodes, const int32_t* __restrict__ conn,
                                                                 const int64_t* __restrict__ inc_ptr,
                                                                 const int32_t* __restrict__ inc,
                                                                 int32_t* __restrict__ deg, int32_t* __restrict__ err) {
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t n = (int64_t)blockIdx.x * kPatWaves + w;
    if (n >= n_nodes) return;
    const int64_t k0 = inc_ptr[n], cnt = inc_ptr[n + 1] - k0;
    int c;
    if (cnt <= 8) {
        const int kk = lane >> 3, j = lane & 7;
        uint64_t key = ~0ull;
        if (kk < cnt) key = ((uint64_t)(uint32_t)conn[(int64_t)(inc[k0 + kk] >> 3) * 8 + j] << 32) | (uint64_t)lane;
        c = wave_neighbours(key, lane).deg;
    } else {
        int32_t nb[kMaxNbr];
        c = (lane == 0) ? node_neighbours((int32_t)n, conn, inc_ptr, inc, nb) : 0;
    }
    if (lane == 0) {
        if (c < 0) {
            atomicOr(err, ERR_DEGREE);
            c = 0;
        } else if (c == 0) {
            atomicOr(err, ERR_ORPHAN);
        }
        deg[n] = c;
    }
}

// Column indices of node n's three rows and the elem_rank entries of every
// (element, local index) pair that is node n.
__global__ __launch_bounds__(64 * kPatWaves) void node_fill_w(int32_t n_nodes, const int32_t* __restrict__ conn,
                                                               const int64_t* __restrict__ inc_ptr,
                                                               const int32_t* __restrict__ inc,
                                                               const int32_t* __restrict__ row_ptr,
                                                               int32_t* __restrict__ col_idx,
                                                               uint8_t* __restrict__ rank) {
    __shared__ int32_t snb[kPatWaves][kMaxNbr];
    __shared__ int32_t srk[kPatWaves][64];
    __shared__ int32_t sdeg[kPatWaves];
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t n = (int64_t)blockIdx.x * kPatWaves + w;
    if (n >= n_nodes) return;
    const int64_t k0 = inc_ptr[n], k1 = inc_ptr[n + 1], cnt = k1 - k0;
    const int kk = lane >> 3, j = lane & 7;
    int deg;
    if (cnt <= 8) {
        int32_t entry = -1;
        uint64_t key = ~0ull;
        if (kk < cnt) {
            entry = inc[k0 + kk];
            key = ((uint64_t)(uint32_t)conn[(int64_t)(entry >> 3) * 8 + j] << 32) | (uint64_t)lane;
        }
        const WaveNbr r = wave_neighbours(key, lane);
        deg = r.deg;
        if (r.first) snb[w][r.uidx] = r.value;
        if (r.origin >= 0) srk[w][r.origin] = r.uidx;
        wave_sync_lds();
        if (entry >= 0) rank[(int64_t)entry * 8 + j] = (uint8_t)srk[w][lane];
    } else {
        if (lane == 0) {
            int32_t nb[kMaxNbr];
            const int c = node_neighbours((int32_t)n, conn, inc_ptr, inc, nb);
            for (int t = 0; t < c; ++t) snb[w][t] = nb[t];
            sdeg[w] = c;
        }
        wave_sync_lds();
        deg = sdeg[w];
        if (deg <= 0) return;  // reported by the counting call
        for (int64_t c = k0; c < k1; c += 8) {
            if (c + kk < k1) {
                const int32_t entry = inc[c + kk];
                const int32_t v = conn[(int64_t)(entry >> 3) * 8 + j];
                int lo = 0, hi = deg - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (snb[w][mid] < v) lo = mid + 1;
                    else hi = mid;
                }
                rank[(int64_t)entry * 8 + j] = (uint8_t)lo;
            }
        }
    }
    int32_t* row = col_idx + row_ptr[3 * n];
    const int32_t len = 3 * deg;
    for (int u = lane; u < deg; u += 64) {
        const int32_t v = snb[w][u];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) row[a * len + 3 * u + b] = 3 * v + b;
    }
}

__global__ void node_columns(int32_t n_nodes, const int32_t* __restrict__ conn, const int64_t* __restrict__ inc_ptr,
                             const int32_t* __restrict__ inc, const int32_t* __restrict__ row_ptr,
                             int32_t* __restrict__ col_idx) {
    int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    int32_t nb[kMaxNbr];
    const int c = node_neighbours(n, conn, inc_ptr, inc, nb);
    if (c <= 0) return;
    for (int a = 0; a < 3; ++a) {
        int32_t* row = col_idx + row_ptr[3 * n + a];
        for (int k = 0; k < c; ++k) {
            row[3 * k + 0] = 3 * nb[k] + 0;
            row[3 * k + 1] = 3 * nb[k] + 1;
            row[3 * k + 2] = 3 * nb[k] + 2;
        }
    }
}

// node -> conn-entry incidence in ascending order (deterministic assembly)
__global__ void write_incidence(int32_t n_nodes, const int64_t* __restrict__ inc_ptr,
                                const int32_t* __restrict__ inc, int32_t* __restrict__ out_ptr,
                                int32_t* __restrict__ out) {
    const int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n > n_nodes) return;
    out_ptr[n] = (int32_t)inc_ptr[n];
    if (n == n_nodes) return;
    const int64_t b = inc_ptr[n], e = inc_ptr[n + 1];
    for (int64_t k = b; k < e; ++k) {
        const int32_t v = inc[k];
        int64_t p = k;
        while (p > b && out[p - 1] > v) {
            out[p] = out[p - 1];
            --p;
        }
        out[p] = v;
    }
}

__global__ void write_row_ptr(int32_t n_nodes, const int32_t* __restrict__ deg, const int64_t* __restrict__ dscan,
                              int32_t* __restrict__ row_ptr) {
    int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n > n_nodes) return;
    if (n == n_nodes) {
        row_ptr[3 * (int64_t)n_nodes] = (int32_t)(9 * dscan[n_nodes]);
        return;
    }
    const int64_t base = 9 * dscan[n];
    const int32_t dg = deg[n];
    for (int a = 0; a < 3; ++a) row_ptr[3 * (int64_t)n + a] = (int32_t)(base + 3 * a * dg);
}

// ---- exclusive scan of int32 -> int64 (out has n+1 entries; out[n] = total)

__global__ void scan_block_sums(const int32_t* __restrict__ in, int64_t n, int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) s += in[i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0];
}

// single workgroup: exclusive scan of nb block sums in place
__global__ void scan_block_offsets(int64_t* __restrict__ bsum, int64_t nb) {
    __shared__ int64_t sh[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    int64_t s = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) s += bsum[b0 + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 thread totals
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = ((int)threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = sh[threadIdx.x] - s;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) {
            const int64_t v = bsum[b0 + k];
            bsum[b0 + k] = run;
            run += v;
        }
}

__global__ void scan_apply(const int32_t* __restrict__ in, int64_t n, const int64_t* __restrict__ boff,
                           int64_t* __restrict__ out) {
    __shared__ int64_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int64_t t = ((int)threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = boff[blockIdx.x] + sh[threadIdx.x] - s;
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
        if (base + k == n - 1) out[n] = run;
    }
}

hipError_t exclusive_scan(const int32_t* in, int64_t n, int64_t* out, int64_t* bsum, hipStream_t s) {
    if (n == 0) {
        return zero_bytes(out, sizeof(int64_t), s);
    }
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(scan_block_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, bsum);
    hipLaunchKernelGGL(scan_block_offsets, dim3(1), dim3(1024), 0, s, bsum, nb);
    hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, bsum, out);
    return hipGetLastError();
}

struct PatternWs {
    int32_t* cnt;      // [n_nodes]
    int64_t* inc_ptr;  // [n_nodes + 1]
    int32_t* fillc;    // [n_nodes]
    int32_t* inc;      // [8 n_elems]
    int32_t* deg;      // [n_nodes]
    int64_t* dscan;    // [n_nodes + 1]
    int64_t* bsum;     // scan block sums
    int32_t* err;      // [1]
};

template <typename C>
void carve_pattern(C& c, int32_t n_nodes, int32_t n_elems, PatternWs* w) {
    const size_t nb = ((size_t)n_nodes + kScanChunk) / kScanChunk + 1;
    auto cnt = c.template take<int32_t>((size_t)n_nodes + 1);
    auto ip = c.template take<int64_t>((size_t)n_nodes + 1);
    auto fc = c.template take<int32_t>((size_t)n_nodes + 1);
    auto inc = c.template take<int32_t>((size_t)n_elems * 8 + 1);
    auto deg = c.template take<int32_t>((size_t)n_nodes + 1);
    auto ds = c.template take<int64_t>((size_t)n_nodes + 1);
    auto bs = c.template take<int64_t>(nb);
    auto er = c.template take<int32_t>(64);
    if (w) *w = PatternWs{cnt, ip, fc, inc, deg, ds, bs, er};
}

// take<> of the counter returns void; adapt so the same carving code runs
struct CountAdapter {
    WsCounter cnt;
    template <typename T>
    T* take(size_t n) {
        cnt.take<T>(n);
        return nullptr;
    }
};

// Steps 1-2 (+ degree scan): incidence, neighbour counts, row_ptr.
int build_incidence(const fem_mesh* m, const PatternWs& w, hipStream_t s) {
    const int64_t ne8 = (int64_t)m->n_elems * 8;
    const int32_t nn = m->n_nodes;
    FEM_HIP_CHECK(zero_bytes(w.cnt, sizeof(int32_t) * ((size_t)nn + 1), s));
    FEM_HIP_CHECK(zero_bytes(w.fillc, sizeof(int32_t) * ((size_t)nn + 1), s));
    FEM_HIP_CHECK(zero_bytes(w.err, sizeof(int32_t), s));
    const int T = 256;
    if (ne8 > 0)
        hipLaunchKernelGGL(count_incidence, dim3((unsigned)((ne8 + T - 1) / T)), dim3(T), 0, s, m->conn, ne8, nn,
                           w.cnt, w.err);
    FEM_HIP_CHECK(exclusive_scan(w.cnt, nn, w.inc_ptr, w.bsum, s));
    if (ne8 > 0)
        hipLaunchKernelGGL(fill_incidence, dim3((unsigned)((ne8 + T - 1) / T)), dim3(T), 0, s, m->conn, ne8, nn,
                           w.inc_ptr, w.fillc, w.inc);
    if (nn > 0)
        hipLaunchKernelGGL(node_degree_w, dim3((unsigned)((nn + kPatWaves - 1) / kPatWaves)), dim3(64 * kPatWaves), 0,
                           s, nn, m->conn, w.inc_ptr, w.inc, w.deg, w.err);
    FEM_HIP_CHECK(exclusive_scan(w.deg, nn, w.dscan, w.bsum, s));
    FEM_HIP_CHECK(hipGetLastError());
    return FEM_OK;
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" size_t fem_csr_workspace_bytes(int32_t n_nodes, int32_t n_elems) {
    if (n_nodes < 0 || n_elems < 0) return 0;
    CountAdapter c;
    carve_pattern(c, n_nodes, n_elems, (PatternWs*)nullptr);
    return c.cnt.used + 256;
}

extern "C" int fem_csr_pattern(const fem_mesh* mesh, fem_csr* csr, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!mesh || !csr) return set_error(FEM_EINVAL, "fem_csr_pattern: mesh and csr must not be NULL");
    if (mesh->n_nodes < 0 || mesh->n_elems < 0)
        return set_error(FEM_EINVAL, "fem_csr_pattern: negative sizes");
    if ((mesh->n_elems > 0 && !mesh->conn) || !csr->row_ptr)
        return set_error(FEM_EINVAL, "fem_csr_pattern: conn and row_ptr must not be NULL");
    if ((int64_t)mesh->n_nodes * 3 >= INT32_MAX || (int64_t)mesh->n_elems * 8 >= INT32_MAX)
        return set_error(FEM_EOVERFLOW, "fem_csr_pattern: 3*n_nodes or 8*n_elems does not fit in int32");
    hipStream_t s = (hipStream_t)stream;
    const size_t need = fem_csr_workspace_bytes(mesh->n_nodes, mesh->n_elems);
    if (!ws || ws_bytes < need)
        return set_error(FEM_ENOMEM, "fem_csr_pattern: workspace of %zu bytes required, %zu given", need, ws_bytes);
    WsCarver c(ws, ws_bytes);
    PatternWs w;
    carve_pattern(c, mesh->n_nodes, mesh->n_elems, &w);
    csr->n_rows = 3 * mesh->n_nodes;
    int rc = build_incidence(mesh, w, s);
    if (rc) return rc;
    const int T = 256;
    const int32_t nn = mesh->n_nodes;
    if (!csr->col_idx) {
        hipLaunchKernelGGL(write_row_ptr, dim3((unsigned)((nn + 1 + T - 1) / T)), dim3(T), 0, s, nn, w.deg, w.dscan,
                           csr->row_ptr);
        FEM_HIP_CHECK(hipGetLastError());
        int64_t total = 0;
        int32_t err = 0;
        FEM_HIP_CHECK(hipMemcpyAsync(&total, w.dscan + nn, sizeof total, hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipMemcpyAsync(&err, w.err, sizeof err, hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipStreamSynchronize(s));
        if (err & ERR_RANGE) return set_error(FEM_EMESH, "fem_csr_pattern: node index out of range in conn");
        if (err & ERR_DEGREE) return set_error(FEM_EMESH, "fem_csr_pattern: a node has more than 64 neighbours");
        if (err & ERR_ORPHAN) return set_error(FEM_EMESH, "fem_csr_pattern: a node belongs to no element");
        if (9 * total >= (int64_t)INT32_MAX)
            return set_error(FEM_EOVERFLOW, "fem_csr_pattern: nnz = %lld does not fit in int32", (long long)(9 * total));
        csr->nnz = 9 * total;
        return FEM_OK;
    }
    if (nn > 0) {
        if (csr->elem_rank)
            hipLaunchKernelGGL(node_fill_w, dim3((unsigned)((nn + kPatWaves - 1) / kPatWaves)), dim3(64 * kPatWaves),
                               0, s, nn, mesh->conn, w.inc_ptr, w.inc, csr->row_ptr, csr->col_idx, csr->elem_rank);
        else
            hipLaunchKernelGGL(node_columns, dim3((unsigned)((nn + T - 1) / T)), dim3(T), 0, s, nn, mesh->conn,
                               w.inc_ptr, w.inc, csr->row_ptr, csr->col_idx);
    }
    if (csr->node_elem_ptr && csr->node_elem)
        hipLaunchKernelGGL(write_incidence, dim3((unsigned)((nn + 1 + T - 1) / T)), dim3(T), 0, s, nn, w.inc_ptr,
                           w.inc, csr->node_elem_ptr, csr->node_elem);
    FEM_HIP_CHECK(hipGetLastError());
    return FEM_OK;
}
