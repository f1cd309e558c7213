// aux.hip -- small elementwise / reduction kernels: residue validation, plaintext bound, zero
// fill, and the test-only CKKS helpers (coefficient encoding, encryption/decryption combine).
#include "common.hpp"
#include "launch.hpp"

namespace hlb {

constexpr int kAuxThreads = 256;

static int aux_grid(int64_t count) {
    const int64_t per = (int64_t)kAuxThreads * 8;
    int64_t g = (count + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65535) g = 65535;
    return (int)g;
}

// Smallest linear index (row * cols + col) of an entry >= q; the atomic min runs only on
// offending entries, so the common all-valid case does no atomics.
__global__ void validate_kernel(const uint64_t *__restrict__ X, int64_t rows, int64_t cols, int64_t ld,
                                uint64_t q, unsigned long long *first_bad) {
    const int64_t total = rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols, c = i - r * cols;
        if (X[r * ld + c] >= q) atomicMin(first_bad, (unsigned long long)i);
    }
}

__global__ void absmax_kernel(const int64_t *__restrict__ P, int64_t m, int64_t k, int64_t ld,
                              unsigned long long *out) {
    __shared__ unsigned long long red[kAuxThreads];
    unsigned long long best = 0;
    const int64_t total = m * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / k, c = i - r * k;
        const int64_t v = P[r * ld + c];
        const unsigned long long a = v < 0 ? (unsigned long long)0 - (unsigned long long)v
                                           : (unsigned long long)v;
        best = a > best ? a : best;
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = kAuxThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, red[0]);
}

// `value` in a rows x cols block of 64-bit words (row stride ld): zeros for the outputs of a
// product over k = 0, start values of the reduction counters.  A kernel rather than a memset,
// so that a caller may capture the call in a graph.
__global__ void fill_kernel(uint64_t *__restrict__ C, int64_t rows, int64_t cols, int64_t ld, uint64_t value) {
    const int64_t total = rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols, c = i - r * cols;
        C[r * ld + c] = value;
    }
}

// The paper's rounding floor(x + 1/2) of delta * M (Section 2 notation; coefficient encoding).
__global__ void encode_kernel(const double *__restrict__ M, int64_t count, double delta, int64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int64_t)__builtin_floor(M[i] * delta + 0.5);
}

__device__ __forceinline__ uint64_t residue_of_signed(int64_t v, uint64_t q) {
    if (v >= 0) return (uint64_t)v % q;
    const uint64_t r = ((uint64_t)0 - (uint64_t)v) % q;
    return r == 0 ? 0 : q - r;
}

__global__ void residues_kernel(const int64_t *__restrict__ v, int64_t count, uint64_t q, uint64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = residue_of_signed(v[i], q);
}

// out = (sign * AS + E) mod q with AS a residue, E either signed (Es) or a residue (Eu).
__global__ void combine_kernel(const uint64_t *__restrict__ AS, const int64_t *__restrict__ Es,
                               const uint64_t *__restrict__ Eu, int sign, int64_t count, uint64_t q,
                               uint64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t a = AS[i];
        if (sign < 0) a = a == 0 ? 0 : q - a;
        const uint64_t e = Es ? residue_of_signed(Es[i], q) : Eu[i];
        out[i] = addmod(a, e, q);
    }
}

// Rescale by the last prime q: c = centred residue of x mod q (ties upward), then
// y_l = (x_l - c) * q^{-1} mod q_l for l < L-1.  qinv_l = q^{-1} mod q_l with its Shoup
// companion; all moduli < 2^52.
__global__ void rescale_kernel(const uint64_t *__restrict__ X, int64_t count, RescaleConsts rc, uint64_t *Y) {
    const uint64_t q = rc.q[rc.L - 1];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t r = X[(int64_t)(rc.L - 1) * count + i];
        const bool up = 2 * r >= q;  // c = r - q when r/q >= 1/2 (round half up), else c = r
        for (int l = 0; l < rc.L - 1; ++l) {
            const uint64_t ql = rc.q[l];
            // c mod ql: r mod ql, minus q mod ql when c = r - q
            uint64_t cm = r % ql;
            if (up) cm = cm >= rc.q_mod[l] ? cm - rc.q_mod[l] : cm + ql - rc.q_mod[l];
            const uint64_t xl = X[(int64_t)l * count + i];
            const uint64_t d = xl >= cm ? xl - cm : xl + ql - cm;
            Y[(int64_t)l * count + i] = mulmod_shoup(d, rc.qinv[l], rc.qinv_shoup[l], ql);
        }
    }
}

hipError_t launch_rescale(const uint64_t *X, int64_t count, const RescaleConsts &rc, uint64_t *Y, hipStream_t s) {
    hipLaunchKernelGGL(rescale_kernel, dim3(aux_grid(count)), dim3(kAuxThreads), 0, s, X, count, rc, Y);
    return hipGetLastError();
}

hipError_t launch_validate(const uint64_t *X, int64_t rows, int64_t cols, int64_t ld, uint64_t q,
                           unsigned long long *first_bad, hipStream_t s) {
    hipLaunchKernelGGL(validate_kernel, dim3(aux_grid(rows * cols)), dim3(kAuxThreads), 0, s, X, rows,
                       cols, ld, q, first_bad);
    return hipGetLastError();
}

hipError_t launch_absmax(const int64_t *P, int64_t m, int64_t k, int64_t ld, unsigned long long *out,
                         hipStream_t s) {
    hipLaunchKernelGGL(absmax_kernel, dim3(aux_grid(m * k)), dim3(kAuxThreads), 0, s, P, m, k, ld, out);
    return hipGetLastError();
}

hipError_t launch_fill(uint64_t *C, int64_t rows, int64_t cols, int64_t ld, uint64_t value, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(aux_grid(rows * cols)), dim3(kAuxThreads), 0, s, C, rows, cols, ld, value);
    return hipGetLastError();
}

hipError_t launch_zero(uint64_t *C, int64_t rows, int64_t cols, int64_t ld, hipStream_t s) {
    return launch_fill(C, rows, cols, ld, 0, s);
}

hipError_t launch_encode(const double *M, int64_t count, double delta, int64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(encode_kernel, dim3(aux_grid(count)), dim3(kAuxThreads), 0, s, M, count, delta, out);
    return hipGetLastError();
}

hipError_t launch_residues_of_signed(const int64_t *v, int64_t count, uint64_t q, uint64_t *out,
                                     hipStream_t s) {
    hipLaunchKernelGGL(residues_kernel, dim3(aux_grid(count)), dim3(kAuxThreads), 0, s, v, count, q, out);
    return hipGetLastError();
}

hipError_t launch_combine(const uint64_t *AS, const int64_t *Es, const uint64_t *Eu, int sign,
                          int64_t count, uint64_t q, uint64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3(aux_grid(count)), dim3(kAuxThreads), 0, s, AS, Es, Eu, sign,
                       count, q, out);
    return hipGetLastError();
}

}  // namespace hlb
