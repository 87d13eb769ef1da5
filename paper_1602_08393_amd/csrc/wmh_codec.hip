// b-bit signatures.  The hash values are geometric with mean 1/s (Theorem 2), so they are small
// with high probability (Corollary 1) and a few bits per value hold them (the paper reports
// 5-9 bits on its datasets, Table 3).  Layout: f = floor(32 / b) fields per 32-bit word; field
// i of a row sits in word i / f at bit (i mod f) * b; a row has W = ceil(k / f) words; unused
// bits and fields are 0; values above 2^b - 1 are stored as 2^b - 1 (saturated).
//
// Collisions are counted on the packed words: xor two words and count the zero fields with a
// carry-free test (per field, (d & low) + low sets the field's top bit iff a low bit of d is
// set; or-ing d covers the top bit itself), so one word compares f hashes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "wmh_internal.h"

namespace wmh {

namespace {

__device__ __forceinline__ uint32_t lane() { return threadIdx.x & (kWave - 1u); }

struct FieldMasks {
    uint32_t low;   // the low b-1 bits of every used field
    uint32_t high;  // the top bit of every used field
};

__host__ __device__ inline FieldMasks field_masks(uint32_t bits)
{
    const uint32_t f = 32u / bits;
    FieldMasks m{0u, 0u};
    for (uint32_t i = 0; i < f; ++i) {
        m.high |= 1u << (i * bits + bits - 1u);
        m.low |= ((1u << (bits - 1u)) - 1u) << (i * bits);
    }
    return m;
}

__device__ __forceinline__ uint32_t zero_fields(uint32_t d, FieldMasks m)
{
    return __builtin_popcount(~(((d & m.low) + m.low) | d) & m.high);
}

// One thread per output word; saturated values counted per workgroup, one atomic each.
__global__ __launch_bounds__(256) void pack_kernel(const uint16_t *__restrict__ sig,
                                                   uint64_t n_rows, uint32_t k, uint32_t bits,
                                                   uint32_t words, uint32_t *__restrict__ packed,
                                                   unsigned long long *saturated)
{
    __shared__ uint32_t part[256 / kWave];
    const uint32_t f = 32u / bits;
    const uint32_t top = (1u << bits) - 1u;
    const uint64_t total = n_rows * words;
    uint32_t sat = 0;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = idx / words;
        const uint32_t w = (uint32_t)(idx - r * words);
        const uint32_t i0 = w * f, i1 = min(k, i0 + f);
        const uint16_t *row = sig + r * k;
        uint32_t word = 0;
        for (uint32_t i = i0; i < i1; ++i) {
            const uint32_t v = row[i];
            sat += v > top;
            word |= min(v, top) << ((i - i0) * bits);
        }
        packed[idx] = word;
    }
    for (int off = 32; off > 0; off >>= 1) sat += __shfl_xor(sat, off);
    if (lane() == 0) part[threadIdx.x / kWave] = sat;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (uint32_t w = 0; w < blockDim.x / kWave; ++w) s += part[w];
        if (s) atomicAdd(saturated, s);
    }
}

__global__ __launch_bounds__(256) void unpack_kernel(const uint32_t *__restrict__ packed,
                                                     uint64_t n_rows, uint32_t k, uint32_t bits,
                                                     uint32_t words, uint16_t *__restrict__ sig)
{
    const uint32_t f = 32u / bits;
    const uint32_t top = (1u << bits) - 1u;
    const uint64_t total = n_rows * words;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = idx / words;
        const uint32_t w = (uint32_t)(idx - r * words);
        const uint32_t i0 = w * f, i1 = min(k, i0 + f);
        const uint32_t word = packed[idx];
        uint16_t *row = sig + r * k;
        for (uint32_t i = i0; i < i1; ++i) row[i] = (uint16_t)((word >> ((i - i0) * bits)) & top);
    }
}

__global__ __launch_bounds__(256) void max_kernel(const uint16_t *__restrict__ sig, uint64_t n,
                                                  uint32_t *max_value)
{
    uint32_t m = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        m = max(m, (uint32_t)sig[i]);
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if (lane() == 0 && m) atomicMax(max_value, m);
}

constexpr int kTile = 64;           // rows of A (and of B) per workgroup
constexpr int kChunkWords = 32;     // packed words per staged chunk
constexpr int kPitch = kChunkWords + 1;

// All pairs: a 64 x 64 block of pairs per workgroup, a 4 x 4 register tile per thread.
// Words past a row's end pad A with 0 and B with all ones, so they never count; the unused
// fields of a row's last word are 0 in both and are taken off at the end.
__global__ __launch_bounds__(256) void packed_collide_kernel(const uint32_t *__restrict__ A,
                                                             uint64_t na,
                                                             const uint32_t *__restrict__ B,
                                                             uint64_t nb, uint32_t words,
                                                             uint32_t pad_fields, FieldMasks fm,
                                                             uint32_t *__restrict__ counts)
{
    __shared__ uint32_t sa[kTile * kPitch];
    __shared__ uint32_t sb[kTile * kPitch];
    const uint64_t a0 = (uint64_t)blockIdx.y * kTile;
    const uint64_t b0 = (uint64_t)blockIdx.x * kTile;
    const uint32_t tx = threadIdx.x & 15u, ty = threadIdx.x >> 4;
    uint32_t acc[4][4] = {};
    for (uint32_t w0 = 0; w0 < words; w0 += kChunkWords) {
        for (uint32_t i = threadIdx.x; i < kTile * kChunkWords; i += blockDim.x) {
            const uint32_t r = i / kChunkWords, w = i - r * kChunkWords;
            const uint32_t wi = w0 + w;
            uint32_t va = 0u, vb = ~0u;
            if (wi < words && a0 + r < na) va = A[(a0 + r) * words + wi];
            if (wi < words && b0 + r < nb) vb = B[(b0 + r) * words + wi];
            sa[r * kPitch + w] = va;
            sb[r * kPitch + w] = vb;
        }
        __syncthreads();
#pragma unroll 4
        for (int w = 0; w < kChunkWords; ++w) {
            uint32_t ra[4], rb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ra[i] = sa[(ty + 16 * i) * kPitch + w];
                rb[i] = sb[(tx + 16 * i) * kPitch + w];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][q] += zero_fields(ra[i] ^ rb[q], fm);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t a = a0 + ty + 16 * i;
        if (a >= na) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t b = b0 + tx + 16 * q;
            if (b < nb) counts[a * nb + b] = acc[i][q] - pad_fields;
        }
    }
}

// Row-aligned pairs: one wavefront per pair.
__global__ __launch_bounds__(256) void packed_estimate_kernel(const uint32_t *__restrict__ A,
                                                              const uint32_t *__restrict__ B,
                                                              uint64_t n_pairs, uint32_t words,
                                                              uint32_t pad_fields, uint32_t k,
                                                              FieldMasks fm, uint32_t *count,
                                                              double *jhat)
{
    const uint32_t waves = blockDim.x / kWave;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    for (uint64_t p = (uint64_t)blockIdx.x * waves + wave; p < n_pairs;
         p += (uint64_t)gridDim.x * waves) {
        uint32_t n = 0;
        for (uint32_t w = lane(); w < words; w += kWave)
            n += zero_fields(A[p * words + w] ^ B[p * words + w], fm);
        for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off);
        n -= pad_fields;
        if (lane() == 0) {
            if (count) count[p] = n;
            if (jhat) jhat[p] = (double)n / (double)k;
        }
    }
}

uint32_t grid_for(uint64_t items)
{
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((items + 255) / 256, 65536));
}

}  // namespace

uint32_t pack_words(uint32_t k, uint32_t bits)
{
    if (bits < 1 || bits > 16 || k == 0) return 0;
    const uint32_t f = 32u / bits;
    return (k + f - 1) / f;
}

hipError_t launch_pack(const uint16_t *sig, uint64_t n_rows, uint32_t k, uint32_t bits,
                       uint32_t *packed, unsigned long long *saturated, hipStream_t stream)
{
    const uint32_t words = pack_words(k, bits);
    pack_kernel<<<grid_for(n_rows * words), 256, 0, stream>>>(sig, n_rows, k, bits, words, packed,
                                                              saturated);
    return hipGetLastError();
}

hipError_t launch_unpack(const uint32_t *packed, uint64_t n_rows, uint32_t k, uint32_t bits,
                         uint16_t *sig, hipStream_t stream)
{
    const uint32_t words = pack_words(k, bits);
    unpack_kernel<<<grid_for(n_rows * words), 256, 0, stream>>>(packed, n_rows, k, bits, words, sig);
    return hipGetLastError();
}

hipError_t launch_sig_max(const uint16_t *sig, uint64_t n, uint32_t *max_value, hipStream_t stream)
{
    max_kernel<<<grid_for(n), 256, 0, stream>>>(sig, n, max_value);
    return hipGetLastError();
}

hipError_t launch_packed_collisions(const uint32_t *A, uint64_t na, const uint32_t *B, uint64_t nb,
                                    uint32_t k, uint32_t bits, uint32_t *counts, hipStream_t stream)
{
    if (na == 0 || nb == 0) return hipSuccess;
    const uint64_t gx = (nb + kTile - 1) / kTile, gy = (na + kTile - 1) / kTile;
    if (gx > 0x7FFFFFFFull || gy > 65535ull) return hipErrorInvalidValue;
    const uint32_t words = pack_words(k, bits);
    const uint32_t pad = words * (32u / bits) - k;
    packed_collide_kernel<<<dim3((uint32_t)gx, (uint32_t)gy), 256, 0, stream>>>(
        A, na, B, nb, words, pad, field_masks(bits), counts);
    return hipGetLastError();
}

hipError_t launch_packed_estimate(const uint32_t *A, const uint32_t *B, uint64_t n_pairs,
                                  uint32_t k, uint32_t bits, uint32_t *count, double *jhat,
                                  hipStream_t stream)
{
    if (n_pairs == 0) return hipSuccess;
    const uint32_t words = pack_words(k, bits);
    const uint32_t pad = words * (32u / bits) - k;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((n_pairs + 3) / 4, 65536);
    packed_estimate_kernel<<<grid, 256, 0, stream>>>(A, B, n_pairs, words, pad, k,
                                                     field_masks(bits), count, jhat);
    return hipGetLastError();
}

}  // namespace wmh
