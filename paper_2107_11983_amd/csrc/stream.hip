// Streamed output (Implementation details, input and output: the engine
// fills one buffer while the other is written out, double buffering).  The
// batch runs in chunks of queries; each chunk's paths are packed on the
// device into one contiguous run of entries with per-query offsets, copied
// by DMA into one of two pinned host buffers, and handed to the caller's
// function while the next chunk walks.  The device side holds two sets of
// chunk buffers, so chunk i+1 walks while chunk i is packed and copied.
#include <hip/hip_runtime.h>

#include <errno.h>
#include <unistd.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "trw_device.hpp"
#include "trw_internal.hpp"

namespace trw {
namespace {

constexpr uint32_t kScanItems = 4;                       // items per thread in the block scan
constexpr uint32_t kScanBlock = 256 * kScanItems;        // items per workgroup

inline size_t up256(size_t x) { return (x + 255) / 256 * 256; }

// Layout of one device chunk set and of one host chunk set (offsets in bytes).
struct ChunkLayout {
    size_t paths, lengths, status, counts, offsets, entries, block_sums, total;
};

ChunkLayout device_layout(uint32_t chunk, uint64_t stride, uint32_t max_len) {
    ChunkLayout l{};
    size_t o = 0;
    l.paths = o;      o += up256(sizeof(int32_t) * (size_t)chunk * stride);
    l.lengths = o;    o += up256(sizeof(uint32_t) * (size_t)chunk);
    l.status = o;     o += up256((size_t)chunk);
    l.counts = o;     o += up256(sizeof(uint64_t) * (size_t)chunk);
    l.offsets = o;    o += up256(sizeof(uint64_t) * ((size_t)chunk + 1));
    l.entries = o;    o += up256(sizeof(int32_t) * (size_t)chunk * ((size_t)max_len + 1));
    l.block_sums = o; o += up256(sizeof(uint64_t) * (((size_t)chunk + kScanBlock - 1) / kScanBlock + 1));
    l.total = o;
    return l;
}

ChunkLayout host_layout(uint32_t chunk, uint32_t max_len) {
    ChunkLayout l{};
    size_t o = 0;
    l.lengths = o;  o += up256(sizeof(uint32_t) * (size_t)chunk);
    l.status = o;   o += up256((size_t)chunk);
    l.offsets = o;  o += up256(sizeof(uint64_t) * ((size_t)chunk + 1));
    l.entries = o;  o += up256(sizeof(int32_t) * (size_t)chunk * ((size_t)max_len + 1));
    l.total = o;
    return l;
}

// Entries per query (its path, or nothing for a bad source), scanned within
// each workgroup of kScanBlock queries; counts[q] gets the workgroup-local
// exclusive offset and block_sums[b] the workgroup's total.
__global__ void __launch_bounds__(256) k_pack_scan(const uint32_t *__restrict__ lengths,
                                                  const uint8_t *__restrict__ status, uint32_t nq,
                                                  uint64_t *__restrict__ counts, uint64_t *__restrict__ block_sums) {
    __shared__ uint64_t wave_tot[4];
    const uint32_t base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    uint64_t c[kScanItems];
    uint64_t mine = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
        const uint32_t q = base + j;
        c[j] = (q < nq && status[q] != ST_BAD_SOURCE) ? (uint64_t)lengths[q] + 1 : 0;
        mine += c[j];
    }
    uint64_t incl = mine;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == 63) wave_tot[wv] = incl;
    __syncthreads();
    uint64_t before = 0;
    for (uint32_t k = 0; k < wv; ++k) before += wave_tot[k];
    uint64_t run = before + incl - mine;
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
        const uint32_t q = base + j;
        if (q < nq) counts[q] = run;
        run += c[j];
    }
    if (threadIdx.x == 255) block_sums[blockIdx.x] = before + incl;
}

// Exclusive scan of the workgroup totals, in place; the grand total goes to
// offsets[nq].  One workgroup, sequential over the (few) totals per thread.
__global__ void __launch_bounds__(256) k_pack_block_sums(uint64_t *__restrict__ block_sums, uint32_t nblocks,
                                                        uint64_t *__restrict__ offsets, uint32_t nq) {
    __shared__ uint64_t wave_tot[4];
    const uint32_t per = (nblocks + 255) / 256;
    const uint32_t lo = threadIdx.x * per, hi = min(nblocks, lo + per);
    uint64_t mine = 0;
    for (uint32_t b = lo; b < hi; ++b) mine += block_sums[b];
    uint64_t incl = mine;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == 63) wave_tot[wv] = incl;
    __syncthreads();
    uint64_t before = 0;
    for (uint32_t k = 0; k < wv; ++k) before += wave_tot[k];
    uint64_t run = before + incl - mine;
    for (uint32_t b = lo; b < hi; ++b) {
        const uint64_t s = block_sums[b];
        block_sums[b] = run;
        run += s;
    }
    if (threadIdx.x == 255) offsets[nq] = before + incl;
}

// Final offsets, and each query's path copied into the packed run.
__global__ void __launch_bounds__(256) k_pack_copy(const int32_t *__restrict__ paths, uint64_t stride,
                                                  const uint32_t *__restrict__ lengths,
                                                  const uint8_t *__restrict__ status, uint32_t nq,
                                                  const uint64_t *__restrict__ counts,
                                                  const uint64_t *__restrict__ block_sums,
                                                  uint64_t *__restrict__ offsets, int32_t *__restrict__ entries) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const uint64_t at = block_sums[q / kScanBlock] + counts[q];
    offsets[q] = at;
    if (status[q] == ST_BAD_SOURCE) return;
    const uint32_t n = lengths[q] + 1;
    const int32_t *src = paths + (uint64_t)q * stride;
    for (uint32_t i = 0; i < n; ++i) entries[at + i] = src[i];
}

trw_status sfail(trw_status st, const std::string &m) {
    set_error(m);
    return st;
}

}  // namespace
}  // namespace trw

using namespace trw;

extern "C" {

trw_status trw_walk_stream_bytes(trw_graph g, const trw_walk_params *p, uint32_t chunk_queries,
                                 size_t *device_bytes, size_t *host_bytes) {
    if (!g || !p || !device_bytes || !host_bytes) return sfail(TRW_E_INVALID, "graph / params / bytes is NULL");
    if (chunk_queries == 0) return sfail(TRW_E_INVALID, "chunk_queries must be >= 1");
    size_t walk_ws = 0;
    trw_status st = trw_walk_workspace_bytes(g, p, chunk_queries, TRW_M_PERSISTENT, &walk_ws);
    if (st != TRW_OK) return st;
    const uint64_t stride = ((uint64_t)p->max_len + 1 + 15) / 16 * 16;
    *device_bytes = 2 * device_layout(chunk_queries, stride, p->max_len).total + up256(walk_ws);
    *host_bytes = 2 * host_layout(chunk_queries, p->max_len).total;
    return TRW_OK;
}

trw_status trw_walk_stream(trw_graph g, trw_table table, const trw_walk_params *p, const int32_t *d_sources,
                           uint64_t nq, uint64_t qid_base, uint32_t chunk_queries, const trw_tuning *tuning,
                           void *d_ws, size_t d_ws_bytes, void *h_pinned, size_t h_bytes, trw_chunk_fn fn,
                           void *user, trw_stream_t stream) {
    size_t need_d = 0, need_h = 0;
    trw_status st = trw_walk_stream_bytes(g, p, chunk_queries, &need_d, &need_h);
    if (st != TRW_OK) return st;
    if (!fn) return sfail(TRW_E_INVALID, "fn is NULL");
    if (nq >= (uint64_t(1) << 32)) return sfail(TRW_E_INVALID, "nq must be < 2^32");
    if (nq > 0 && !d_sources) return sfail(TRW_E_INVALID, "sources is NULL");
    if (!d_ws || d_ws_bytes < need_d || (reinterpret_cast<uintptr_t>(d_ws) & 255))
        return sfail(TRW_E_INVALID, "device workspace NULL, too small or not 256-byte aligned");
    if (!h_pinned || h_bytes < need_h || (reinterpret_cast<uintptr_t>(h_pinned) & 255))
        return sfail(TRW_E_INVALID, "host buffer NULL, too small or not 256-byte aligned");
    if (nq == 0) return TRW_OK;

    const uint32_t C = chunk_queries;
    const uint64_t stride = ((uint64_t)p->max_len + 1 + 15) / 16 * 16;
    const ChunkLayout dl = device_layout(C, stride, p->max_len);
    const ChunkLayout hl = host_layout(C, p->max_len);
    char *dbase[2] = {static_cast<char *>(d_ws), static_cast<char *>(d_ws) + dl.total};
    char *hbase[2] = {static_cast<char *>(h_pinned), static_cast<char *>(h_pinned) + hl.total};
    void *walk_ws = static_cast<char *>(d_ws) + 2 * dl.total;
    const size_t walk_ws_bytes = need_d - 2 * dl.total;
    auto s = static_cast<hipStream_t>(stream);
    const uint64_t n_chunks = (nq + C - 1) / C;

    hipStream_t copy_s = nullptr;
    hipEvent_t packed[2] = {nullptr, nullptr}, meta[2] = {nullptr, nullptr}, done[2] = {nullptr, nullptr};
    hipError_t e = hipStreamCreateWithFlags(&copy_s, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&packed[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&meta[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming);
    }
    auto cleanup = [&]() {
        for (int i = 0; i < 2; ++i) {
            if (packed[i]) (void)hipEventDestroy(packed[i]);
            if (meta[i]) (void)hipEventDestroy(meta[i]);
            if (done[i]) (void)hipEventDestroy(done[i]);
        }
        if (copy_s) (void)hipStreamDestroy(copy_s);
    };
    if (e != hipSuccess) {
        cleanup();
        return sfail(TRW_E_DEVICE, std::string("stream set-up: ") + hipGetErrorString(e));
    }

    // Walk chunk c into device set c % 2 and pack it (on the caller's stream).
    auto launch_chunk = [&](uint64_t c) -> trw_status {
        const uint64_t lo = c * C;
        const uint32_t n = (uint32_t)std::min<uint64_t>(C, nq - lo);
        char *d = dbase[c & 1];
        auto *paths = reinterpret_cast<int32_t *>(d + dl.paths);
        auto *lengths = reinterpret_cast<uint32_t *>(d + dl.lengths);
        auto *status = reinterpret_cast<uint8_t *>(d + dl.status);
        auto *counts = reinterpret_cast<uint64_t *>(d + dl.counts);
        auto *offsets = reinterpret_cast<uint64_t *>(d + dl.offsets);
        auto *entries = reinterpret_cast<int32_t *>(d + dl.entries);
        auto *block_sums = reinterpret_cast<uint64_t *>(d + dl.block_sums);
        trw_status w = trw_walk(g, table, p, d_sources + lo, n, qid_base + lo, paths, stride, lengths, status,
                                TRW_M_PERSISTENT, tuning, walk_ws, walk_ws_bytes, stream);
        if (w != TRW_OK) return w;
        const uint32_t nb = (n + kScanBlock - 1) / kScanBlock;
        hipLaunchKernelGGL(k_pack_scan, dim3(nb), dim3(256), 0, s, lengths, status, n, counts, block_sums);
        hipLaunchKernelGGL(k_pack_block_sums, dim3(1), dim3(256), 0, s, block_sums, nb, offsets, n);
        hipLaunchKernelGGL(k_pack_copy, dim3((n + 255) / 256), dim3(256), 0, s, paths, stride, lengths, status, n,
                           counts, block_sums, offsets, entries);
        hipError_t le = hipGetLastError();
        if (le == hipSuccess) le = hipEventRecord(packed[c & 1], s);
        if (le != hipSuccess) return sfail(TRW_E_DEVICE, std::string("stream chunk launch: ") + hipGetErrorString(le));
        return TRW_OK;
    };

    trw_status result = launch_chunk(0);
    for (uint64_t c = 0; c < n_chunks && result == TRW_OK; ++c) {
        // The next chunk walks while this one is copied and consumed.  Its
        // device set was last read by the copies of chunk c - 1, which ended
        // before this iteration began.
        if (c + 1 < n_chunks) result = launch_chunk(c + 1);
        if (result != TRW_OK) break;
        const uint32_t n = (uint32_t)std::min<uint64_t>(C, nq - c * C);
        char *d = dbase[c & 1];
        char *h = hbase[c & 1];
        e = hipStreamWaitEvent(copy_s, packed[c & 1], 0);
        if (e == hipSuccess) e = hipMemcpyAsync(h + hl.lengths, d + dl.lengths, sizeof(uint32_t) * n,
                                                hipMemcpyDeviceToHost, copy_s);
        if (e == hipSuccess) e = hipMemcpyAsync(h + hl.status, d + dl.status, n, hipMemcpyDeviceToHost, copy_s);
        if (e == hipSuccess) e = hipMemcpyAsync(h + hl.offsets, d + dl.offsets, sizeof(uint64_t) * ((size_t)n + 1),
                                                hipMemcpyDeviceToHost, copy_s);
        if (e == hipSuccess) e = hipEventRecord(meta[c & 1], copy_s);
        if (e == hipSuccess) e = hipEventSynchronize(meta[c & 1]);
        if (e != hipSuccess) {
            result = sfail(TRW_E_DEVICE, std::string("stream copy: ") + hipGetErrorString(e));
            break;
        }
        const uint64_t total = reinterpret_cast<const uint64_t *>(h + hl.offsets)[n];
        if (total > (uint64_t)n * ((uint64_t)p->max_len + 1)) {
            result = sfail(TRW_E_DEVICE, "stream: packed size out of range");
            break;
        }
        if (total) e = hipMemcpyAsync(h + hl.entries, d + dl.entries, sizeof(int32_t) * total, hipMemcpyDeviceToHost,
                                      copy_s);
        if (e == hipSuccess) e = hipEventRecord(done[c & 1], copy_s);
        if (e == hipSuccess) e = hipEventSynchronize(done[c & 1]);
        if (e != hipSuccess) {
            result = sfail(TRW_E_DEVICE, std::string("stream copy: ") + hipGetErrorString(e));
            break;
        }
        trw_chunk ch{};
        ch.qid_base = qid_base + c * C;
        ch.nq = n;
        ch.lengths = reinterpret_cast<const uint32_t *>(h + hl.lengths);
        ch.status = reinterpret_cast<const uint8_t *>(h + hl.status);
        ch.offsets = reinterpret_cast<const uint64_t *>(h + hl.offsets);
        ch.entries = reinterpret_cast<const int32_t *>(h + hl.entries);
        if (fn(user, &ch) != 0) {
            result = sfail(TRW_E_CANCELLED, "stream stopped by the chunk function");
            break;
        }
    }
    // Leave nothing in flight on the buffers: the caller may free them on return.
    (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(copy_s);
    cleanup();
    return result;
}

// One chunk appended to the file descriptor *(int *)user as a record:
// header {qid_base u64, nq u32, reserved u32}, lengths u32[nq], status u8[nq]
// padded with zeros to a multiple of 8 bytes, offsets u64[nq + 1], entries
// i32[offsets[nq]].  Runs on the stream's calling thread while the next chunk
// walks, so the disk write overlaps the walk (the engine's double buffering).
int trw_chunk_to_fd(void *user, const trw_chunk *c) {
    if (!user || !c) return 1;
    const int fd = *static_cast<const int *>(user);
    auto put = [fd](const void *data, size_t bytes) -> bool {
        const char *q = static_cast<const char *>(data);
        while (bytes > 0) {
            const ssize_t w = ::write(fd, q, bytes);
            if (w < 0 && errno == EINTR) continue;
            if (w <= 0) return false;
            q += w;
            bytes -= (size_t)w;
        }
        return true;
    };
    struct {
        uint64_t qid_base;
        uint32_t nq, reserved;
    } head{c->qid_base, c->nq, 0};
    static const uint8_t zeros[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const size_t pad = (8 - c->nq % 8) % 8;
    const uint64_t n_entries = c->offsets[c->nq];
    return put(&head, sizeof(head)) && put(c->lengths, sizeof(uint32_t) * (size_t)c->nq) &&
                   put(c->status, (size_t)c->nq) && put(zeros, pad) &&
                   put(c->offsets, sizeof(uint64_t) * ((size_t)c->nq + 1)) &&
                   put(c->entries, sizeof(int32_t) * (size_t)n_entries)
               ? 0
               : 1;
}

}  // extern "C"
