// Device-side seeded input generators (SplitMix64 counter streams, Steele,
// Lea and Flood 2014).  Integer streams are bit-identical to datagen's numpy
// functions of the same name.  Test and benchmark infrastructure: generates
// key and value columns only.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t stream_at(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * GAMMA); }

__device__ __forceinline__ uint64_t mulhi64(uint64_t x, uint64_t m) { return __umul64hi(x, m); }

__global__ void k_uniform_keys(uint64_t seed, uint64_t start, uint64_t n, uint64_t d, uint64_t salt,
                               uint64_t* out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = mulhi64(stream_at(seed, start + i), d);
        out[i] = mix64(r ^ salt);
    }
}

// rank = first index of table with table[idx] >= u (numpy searchsorted, side='left')
__global__ void k_zipf_keys(uint64_t seed, uint64_t start, uint64_t n, const uint64_t* table, uint64_t d,
                            uint64_t salt, uint64_t* out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t u = stream_at(seed, start + i);
        uint64_t lo = 0, hi = d;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (table[mid] < u) lo = mid + 1;
            else hi = mid;
        }
        const uint64_t r = lo < d ? lo : d - 1;
        out[i] = mix64(r ^ salt);
    }
}

__global__ void k_uniform_i64(uint64_t seed, uint64_t start, uint64_t n, int64_t lo, uint64_t span, int64_t* out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = (int64_t)mulhi64(stream_at(seed, start + i), span) + lo;
}

// Ranks uniform over [0, d) (no key mixing).
__global__ void k_uniform_ranks(uint64_t seed, uint64_t start, uint64_t n, uint64_t d, int64_t* out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = (int64_t)mulhi64(stream_at(seed, start + i), d);
}

// B column of the segmented input: per-A domain value j of segment g is the
// top 32 bits of mix(g * b_per_a + j) ^ salt.
__global__ void k_segment_b(uint64_t seed, uint64_t n, uint64_t b_per_a, uint64_t salt, const int64_t* seg,
                            int32_t* b) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = mulhi64(stream_at(seed, i), b_per_a);
        const uint64_t code = (uint64_t)seg[i] * b_per_a + j;
        b[i] = (int32_t)(uint32_t)(mix64(code ^ salt) >> 32);
    }
}

// Approximate Zipf ranks over [0, d) by inverting the continuous density
// proportional to x^-s on [1, d+1) (s != 1; s == 1 inverts the log).  Used
// where an exact CDF table of the domain would be too large.
__global__ void k_zipf_approx_keys(uint64_t seed, uint64_t start, uint64_t n, uint64_t d, double s, uint64_t salt,
                                   uint64_t* out) {
    const double dd = (double)d + 1.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const double u = (double)(stream_at(seed, start + i) >> 11) * (1.0 / 9007199254740992.0);
        double x;
        if (fabs(s - 1.0) < 1e-9) {
            x = exp(u * log(dd));
        } else {
            const double a = 1.0 - s;
            x = pow(u * (pow(dd, a) - 1.0) + 1.0, 1.0 / a);
        }
        uint64_t r = (uint64_t)x;
        r = r >= 1 ? r - 1 : 0;
        if (r >= d) r = d - 1;
        out[i] = mix64(r ^ salt);
    }
}

// Standard normal by the Box-Muller transform of two stream values.
__global__ void k_normal_f64(uint64_t seed, uint64_t start, uint64_t n, double* out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a = stream_at(seed, 2 * (start + i)), b = stream_at(seed, 2 * (start + i) + 1);
        const double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);  // (0, 1]
        const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);          // [0, 1)
        out[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

dim3 grid_for(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    if (g == 0) g = 1;
    return dim3((unsigned)g);
}

}  // namespace

extern "C" {

int dg_uniform_keys(uint64_t seed, uint64_t start, uint64_t n, uint64_t d, uint64_t salt, uint64_t* out, void* st) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_uniform_keys, grid_for(n), dim3(256), 0, (hipStream_t)st, seed, start, n, d, salt, out);
    return (int)hipGetLastError();
}
int dg_zipf_keys(uint64_t seed, uint64_t start, uint64_t n, const uint64_t* table, uint64_t d, uint64_t salt,
                 uint64_t* out, void* st) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_zipf_keys, grid_for(n), dim3(256), 0, (hipStream_t)st, seed, start, n, table, d, salt, out);
    return (int)hipGetLastError();
}
int dg_zipf_approx_keys(uint64_t seed, uint64_t start, uint64_t n, uint64_t d, double s, uint64_t salt, uint64_t* out,
                        void* st) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_zipf_approx_keys, grid_for(n), dim3(256), 0, (hipStream_t)st, seed, start, n, d, s, salt, out);
    return (int)hipGetLastError();
}
int dg_uniform_i64(uint64_t seed, uint64_t start, uint64_t n, int64_t lo, uint64_t span, int64_t* out, void* st) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_uniform_i64, grid_for(n), dim3(256), 0, (hipStream_t)st, seed, start, n, lo, span, out);
    return (int)hipGetLastError();
}
int dg_uniform_ranks(uint64_t seed, uint64_t start, uint64_t n, uint64_t d, int64_t* out, void* st) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_uniform_ranks, grid_for(n), dim3(256), 0, (hipStream_t)st, seed, start, n, d, out);
    return (int)hipGetLastError();
}
int dg_segment_b(uint64_t seed, uint64_t n, uint64_t b_per_a, uint64_t salt, const int64_t* seg, int32_t* b,
                 void* st) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_segment_b, grid_for(n), dim3(256), 0, (hipStream_t)st, seed, n, b_per_a, salt, seg, b);
    return (int)hipGetLastError();
}
int dg_normal_f64(uint64_t seed, uint64_t start, uint64_t n, double* out, void* st) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_normal_f64, grid_for(n), dim3(256), 0, (hipStream_t)st, seed, start, n, out);
    return (int)hipGetLastError();
}

}  // extern "C"
