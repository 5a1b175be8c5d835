// Device-wide exclusive prefix sums (reduce, scan the block sums, scan-and-add), used for
// radix-sort offsets, node and group compaction and list offsets.
#include "common.hpp"

namespace tpm {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

template <typename T>
__device__ T wave_incl_scan(T v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan of one value per thread across the block; returns the block total too.
template <typename T>
__device__ T block_excl_scan(T v, T *total)
{
    __shared__ T wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) {
        T s = wsum[i];
        if (i < w) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_reduce(const T *data, size_t n, T *partials)
{
    size_t base = (size_t)blockIdx.x * kTile;
    T s = 0;
    for (int it = 0; it < kItems; ++it) {
        size_t k = base + (size_t)it * kThreads + threadIdx.x;
        if (k < n) s += data[k];
    }
    T tot;
    (void)block_excl_scan(s, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Scan one tile in place (blocked: thread t owns kItems consecutive values) and add the
// scanned block offset (if any).  If total != nullptr and this is the last block, writes the
// grand total.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_tile(T *data, size_t n, const T *offsets,
                                                        T *total)
{
    size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kItems;
    T v[kItems];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = (base + i < n) ? data[base + i] : T(0);
        s += v[i];
    }
    T tot;
    T run = block_excl_scan(s, &tot);
    T off = offsets ? offsets[blockIdx.x] : T(0);
    run += off;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (base + i < n) data[base + i] = run;
        run += v[i];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

template <typename T>
__global__ void k_set(T *p, size_t n, T v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
void scan_rec(T *data, size_t n, T *total, T *tmp, hipStream_t s)
{
    if (n == 0) {
        k_set<T><<<1, 64, 0, s>>>(total, 1, T(0));
        return;
    }
    size_t nb = (n + kTile - 1) / kTile;
    if (nb == 1) {
        k_scan_tile<T><<<1, kThreads, 0, s>>>(data, n, nullptr, total);
        return;
    }
    T *partials = tmp;
    k_reduce<T><<<(unsigned)nb, kThreads, 0, s>>>(data, n, partials);
    scan_rec<T>(partials, nb, total, tmp + nb, s);
    k_scan_tile<T><<<(unsigned)nb, kThreads, 0, s>>>(data, n, partials, nullptr);
}

// Copies up to three runs of words (src0[0..n0), src1[0..n1), src2[0..n2)) into host-mapped
// memory after word 0, then stores `seq` into word 0 with release order at system scope: a
// host thread that sees seq there also sees the words.
__global__ void k_publish(const uint32_t *__restrict__ src0, uint32_t n0,
                          const uint32_t *__restrict__ src1, uint32_t n1,
                          const uint32_t *__restrict__ src2, uint32_t n2, uint32_t *mailbox,
                          uint32_t seq)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t k = 1;
    for (uint32_t i = 0; i < n0; ++i, ++k)
        __hip_atomic_store(&mailbox[k], src0[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (uint32_t i = 0; i < n1; ++i, ++k)
        __hip_atomic_store(&mailbox[k], src1[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (uint32_t i = 0; i < n2; ++i, ++k)
        __hip_atomic_store(&mailbox[k], src2[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mailbox[0], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

} // namespace

// Fills with a kernel rather than hipMemsetAsync so the calls can sit inside a captured graph.
void fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s)
{
    if (!n) return;
    size_t b = (n + 255) / 256;
    k_set<uint32_t><<<(unsigned)(b < 4096 ? b : 4096), 256, 0, s>>>(p, n, v);
}

void fill_u64(uint64_t *p, size_t n, uint64_t v, hipStream_t s)
{
    if (!n) return;
    size_t b = (n + 255) / 256;
    k_set<uint64_t><<<(unsigned)(b < 4096 ? b : 4096), 256, 0, s>>>(p, n, v);
}

size_t scan_tmp_elems(size_t n)
{
    size_t t = 0;
    while (n > (size_t)kTile) {
        n = (n + kTile - 1) / kTile;
        t += n;
    }
    return t + 16;
}

void scan_u32(uint32_t *data, size_t n, uint32_t *total, uint32_t *tmp, hipStream_t s)
{
    scan_rec<uint32_t>(data, n, total, tmp, s);
}

void scan_u64(uint64_t *data, size_t n, uint64_t *total, uint64_t *tmp, hipStream_t s)
{
    scan_rec<uint64_t>(data, n, total, tmp, s);
}

void publish_words(const uint32_t *src0, uint32_t n0, const uint32_t *src1, uint32_t n1,
                   const uint32_t *src2, uint32_t n2, uint32_t *mailbox, uint32_t seq,
                   hipStream_t s)
{
    k_publish<<<1, 64, 0, s>>>(src0, n0, src1, n1, src2, n2, mailbox, seq);
}

} // namespace tpm
