// scan.hip -- device-wide exclusive prefix sum of int32 counts and a fill
// kernel.  Up to SCAN_SMALL elements one workgroup of 1024 lanes scans in
// chunks with a running carry (one launch, which also returns at once when a
// gating flag is clear: the kept-list substeps); longer inputs take three
// launches: per-block scan of 1024 elements (256 lanes x 4), a single-block
// scan of the block totals, and the block-offset add.
#include "common.h"

namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_PER = 4;
constexpr int SCAN_BLOCK = SCAN_T * SCAN_PER;

// block-wide exclusive scan of one int per lane (64-lane waves, LDS for the
// wave totals); returns the block total through *total
__device__ int block_excl_scan(int v, int* total) {
    __shared__ int wsum[SCAN_T / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_T / 64; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_local(const int* __restrict__ in, int* __restrict__ out,
                                                       long long n, int* __restrict__ bsum, const int* run) {
    if (run && !*run) return;
    long long base = (long long)blockIdx.x * SCAN_BLOCK + (long long)threadIdx.x * SCAN_PER;
    int v[SCAN_PER];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int off = block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
        if (base + k < n) out[base + k] = off;
        off += v[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// single block: exclusive scan of nb block totals, in place; total to out[n]
__global__ __launch_bounds__(SCAN_T) void k_scan_bsum(int* __restrict__ bsum, int nb, int* __restrict__ out,
                                                      long long n, const int* run) {
    if (run && !*run) return;
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += SCAN_T) {
        int i = base + threadIdx.x;
        int v = i < nb ? bsum[i] : 0;
        int tot;
        int ex = block_excl_scan(v, &tot);
        int c = carry;
        if (i < nb) bsum[i] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_add(int* __restrict__ out, long long n,
                                                     const int* __restrict__ bsum, const int* run) {
    if (run && !*run) return;
    long long base = (long long)blockIdx.x * SCAN_BLOCK + (long long)threadIdx.x * SCAN_PER;
    int add = bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k)
        if (base + k < n) out[base + k] += add;
}

constexpr long long SCAN_SMALL = 131072;

// One workgroup of 1024 lanes walks the input in chunks of 4096 entries, four
// consecutive entries per lane (coalesced), with a running carry (in place
// allowed: a lane reads its entries before it writes them).
__device__ inline void scan_small_body(const int* in, int* out, long long n) {
    __shared__ int wsum[16];
    __shared__ int carry_s;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (long long base = 0; base < n; base += 4096) {
        const long long i0 = base + 4LL * tid;
        int v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = i0 + k < n ? in[i0 + k] : 0;
        const int sum = (v[0] + v[1]) + (v[2] + v[3]);
        int x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        const int carry = carry_s;
        int off = carry, tot = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            off += w < wid ? wsum[w] : 0;
            tot += wsum[w];
        }
        int run = off + x - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k < n) {
                out[i0 + k] = run;
                run += v[k];
            }
        __syncthreads();
        if (tid == 0) carry_s = carry + tot;
        __syncthreads();
    }
    if (tid == 0) out[n] = carry_s;
}

__global__ __launch_bounds__(1024) void k_scan_small(const int* in, int* out, long long n, const int* run) {
    if (run && !*run) return;
    scan_small_body(in, out, n);
}

// two short scans, one per workgroup
__global__ __launch_bounds__(1024) void k_scan_small2(const int* in0, int* out0, long long n0, const int* in1,
                                                      int* out1, long long n1) {
    if (blockIdx.x == 0) scan_small_body(in0, out0, n0);
    else scan_small_body(in1, out1, n1);
}

__global__ void k_fill_int(int* __restrict__ p, int v, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

size_t psm_scan_tmp_ints(long long n) { return (size_t)((n + SCAN_BLOCK - 1) / SCAN_BLOCK + 1); }

// the three-launch form at any length
static hipError_t scan_blocks(const int* in, int* out, long long n, int* tmp, hipStream_t s, const int* run) {
    int nb = (int)((n + SCAN_BLOCK - 1) / SCAN_BLOCK);
    if (nb < 1) nb = 1;
    k_scan_local<<<nb, SCAN_T, 0, s>>>(in, out, n, tmp, run);
    k_scan_bsum<<<1, SCAN_T, 0, s>>>(tmp, nb, out, n, run);
    k_scan_add<<<nb, SCAN_T, 0, s>>>(out, n, tmp, run);
    return hipGetLastError();
}

hipError_t psm_scan(const int* in, int* out, long long n, int* tmp, hipStream_t s, const int* run) {
    if (n <= SCAN_SMALL) {
        k_scan_small<<<1, 1024, 0, s>>>(in, out, n < 0 ? 0 : n, run);
        return hipGetLastError();
    }
    return scan_blocks(in, out, n, tmp, s, run);
}

// (one workgroup walking a long input is slower than the three-launch form;
// above SCAN_PAIR_ONE each input takes its own scan)
constexpr long long SCAN_PAIR_ONE = 16384;

hipError_t psm_scan2(const int* in0, int* out0, long long n0, const int* in1, int* out1, long long n1, int* tmp,
                     hipStream_t s) {
    if (n0 <= SCAN_PAIR_ONE && n1 <= SCAN_PAIR_ONE) {
        k_scan_small2<<<2, 1024, 0, s>>>(in0, out0, n0 < 0 ? 0 : n0, in1, out1, n1 < 0 ? 0 : n1);
        return hipGetLastError();
    }
    hipError_t e = scan_blocks(in0, out0, n0 < 0 ? 0 : n0, tmp, s, nullptr);
    return e != hipSuccess ? e : scan_blocks(in1, out1, n1 < 0 ? 0 : n1, tmp, s, nullptr);
}

hipError_t psm_fill_int(int* p, int v, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long nb = (n + 255) / 256;
    k_fill_int<<<(unsigned)nb, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}
