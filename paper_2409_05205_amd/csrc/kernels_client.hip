// Client-side element-wise kernels: lifting signed small polynomials to
// residues, c0 encryption (Alg. 1 / Alg. 2 client encryption, the negated
// encryption of i), and decryption of the share sum by scale-and-round in RNS.
//
// Decryption.  For x = CRT(x_l) in [0, Q) and y_l = x_l (Q/q_l)^-1 mod q_l,
// x = sum_l y_l Q/q_l - a Q for an integer a, so t x / Q = sum_l y_l t / q_l - a t
// and round(t x / Q) mod t = round(sum_l y_l t / q_l) mod t.  Each term is split
// exactly as y_l t = h_l q_l + r_l (64-bit integers); the message is
// (sum h_l + round(sum r_l / q_l)) mod t, where only the fractional sum is in
// double precision (error < 2^-48, while the share sum of a valid ciphertext
// sits within Q/(2t) of Delta m, i.e. t x / Q within far less than 1/4 of an integer).

#include "he_kernels.h"

namespace {

__global__ void k_lift_signed(const int32_t *__restrict__ a, uint32_t *__restrict__ out, uint32_t L, uint32_t N,
                              LimbConsts lc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t r = blockIdx.y;      // row
    const int32_t v = a[(size_t)r * N + k];
    for (uint32_t l = 0; l < L; ++l) {
        const uint32_t q = lc.l[l].q;
        const int64_t m = (int64_t)v % (int64_t)q;
        out[((size_t)r * L + l) * N + k] = (uint32_t)(m < 0 ? m + q : m);
    }
}

__global__ void k_mul_bcast(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b, uint32_t *__restrict__ c,
                            uint32_t L, uint32_t N, LimbConsts lc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t rl = blockIdx.y;     // (row, limb)
    const uint32_t l = rl % L;
    const size_t i = (size_t)rl * N + k;
    c[i] = reduce64((uint64_t)a[i] * b[(size_t)l * N + k], lc.l[l]);
}

// out = -(vb + Delta i + e0) mod q_l
__global__ void k_encrypt_combine(const uint32_t *__restrict__ vb, const uint32_t *__restrict__ msg,
                                  const int32_t *__restrict__ e0, uint32_t *__restrict__ out, uint32_t L, uint32_t N,
                                  LimbConsts lc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t rl = blockIdx.y;
    const uint32_t l = rl % L, r = rl / L;
    const LimbConst &c = lc.l[l];
    const size_t i = (size_t)rl * N + k;
    const uint32_t m = msg[(size_t)r * N + k];
    const uint32_t dm = csub(shoup_lazy(m, c.delta, c.delta_sh, c.q), c.q);
    const int32_t e = e0[(size_t)r * N + k];
    const uint32_t er = e >= 0 ? (uint32_t)e : c.q - (uint32_t)(-e);
    uint32_t s = csub(vb[i] + dm, c.q);
    s = csub(s + er, c.q);
    out[i] = s == 0 ? 0u : c.q - s;
}

__global__ void k_decrypt(const uint32_t *__restrict__ x0, const uint32_t *__restrict__ x1, uint32_t *__restrict__ msg,
                          uint32_t L, uint32_t N, LimbConsts lc, DecConsts dc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t r = blockIdx.y;
    const uint64_t t = dc.t;
    uint64_t hsum = 0;
    double frac = 0.0;
    for (uint32_t l = 0; l < L; ++l) {
        const LimbConst &c = lc.l[l];
        const size_t i = ((size_t)r * L + l) * N + k;
        uint32_t x = x0[i];
        if (x1) x = csub(x + x1[i], c.q);
        const uint32_t y = csub(shoup_lazy(x, dc.inv[l], dc.inv_sh[l], c.q), c.q);
        const uint64_t yt = (uint64_t)y * t;
        const uint64_t h = yt / c.q;
        const uint64_t rem = yt - h * c.q;
        hsum += h;
        frac += (double)rem / (double)c.q;
    }
    const uint64_t whole = hsum + (uint64_t)floor(frac + 0.5);
    msg[(size_t)r * N + k] = (uint32_t)(whole % t);
}


// Client masks of the server initialisation (Alg. 1 / Alg. 2): from the
// server's resident operands S[n][l][J][N] (J < K_in: f NTT(rho_j^(n)),
// J >= K_in: f NTT(-Delta fhat_j^(n)), f the layer's per-slot factor) and the
// client's public key NTT(b), the client operands
//   J < K_in : f NTT(p1) = S_J bhat + f NTT(e1),   p1 = rho b + e1
//   J >= K_in: f NTT(p2) = Delta S_{J-K_in} - S_J + f NTT(e2),   p2 = Delta (fhat + rho) + e2
// where E already holds f NTT(e1) / f NTT(e2) and is overwritten with the result.
__global__ void k_mask_combine(const uint32_t *__restrict__ S, const uint32_t *__restrict__ bhat,
                               uint32_t *__restrict__ E, uint32_t K_in, uint32_t L, uint32_t N, LimbConsts lc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t Jtot = 2 * K_in;
    const uint32_t row = blockIdx.y;          // (n, l, J)
    const uint32_t J = row % Jtot;
    const uint32_t l = (row / Jtot) % L;
    const LimbConst c = lc.l[l];
    const size_t i = (size_t)row * N + k;
    uint32_t v;
    if (J < K_in) {
        v = reduce64((uint64_t)S[i] * bhat[(size_t)l * N + k] + E[i], c);
    } else {
        const uint32_t dr = reduce64((uint64_t)S[i - (size_t)K_in * N] * c.delta, c);   // Delta f NTT(rho)
        v = reduce64((uint64_t)dr + (c.q - S[i]) + E[i], c);
    }
    E[i] = v;
}

// E[n][l][J][k] = e[J][n][k] mod q_l: the mask noise of channel n (J < K_in: e1, else e2),
// small signed values, laid out like the resident operands.
__global__ void k_mask_noise(const int32_t *__restrict__ e1, const int32_t *__restrict__ e2, uint32_t *__restrict__ E,
                             uint32_t K_in, uint32_t n_rows, uint32_t L, uint32_t N, LimbConsts lc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t Jtot = 2 * K_in;
    const uint32_t row = blockIdx.y;
    const uint32_t J = row % Jtot;
    const uint32_t l = (row / Jtot) % L;
    const uint32_t n = row / (Jtot * L);
    const uint32_t q = lc.l[l].q;
    const int32_t x = J < K_in ? e1[((size_t)J * n_rows + n) * N + k] : e2[((size_t)(J - K_in) * n_rows + n) * N + k];
    const int64_t r = (int64_t)x % (int64_t)q;
    E[(size_t)row * N + k] = (uint32_t)(r < 0 ? r + q : r);
}
}  // namespace

hipError_t launch_lift_signed(const int32_t *a, uint32_t *out, uint32_t rows, uint32_t L, uint32_t N,
                              const LimbConsts &lc, hipStream_t st) {
    if (!rows) return hipSuccess;
    hipLaunchKernelGGL(k_lift_signed, dim3((N + 255) / 256, rows), dim3(256), 0, st, a, out, L, N, lc);
    return hipGetLastError();
}

hipError_t launch_mul_bcast(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t rows, uint32_t L, uint32_t N,
                            const LimbConsts &lc, hipStream_t st) {
    if (!rows) return hipSuccess;
    hipLaunchKernelGGL(k_mul_bcast, dim3((N + 255) / 256, rows * L), dim3(256), 0, st, a, b, c, L, N, lc);
    return hipGetLastError();
}

hipError_t launch_encrypt_combine(const uint32_t *vb, const uint32_t *msg, const int32_t *e0, uint32_t *out,
                                  uint32_t rows, uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st) {
    if (!rows) return hipSuccess;
    hipLaunchKernelGGL(k_encrypt_combine, dim3((N + 255) / 256, rows * L), dim3(256), 0, st, vb, msg, e0, out, L, N,
                       lc);
    return hipGetLastError();
}

hipError_t launch_decrypt(const uint32_t *x0, const uint32_t *x1, uint32_t *msg, uint32_t rows, uint32_t L, uint32_t N,
                          const LimbConsts &lc, const DecConsts &dc, hipStream_t st) {
    if (!rows) return hipSuccess;
    hipLaunchKernelGGL(k_decrypt, dim3((N + 255) / 256, rows), dim3(256), 0, st, x0, x1, msg, L, N, lc, dc);
    return hipGetLastError();
}

hipError_t launch_mask_noise(const int32_t *e1, const int32_t *e2, uint32_t *E, uint32_t K_in, uint32_t n_rows,
                             uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st) {
    dim3 grid((N + 255) / 256, n_rows * L * 2 * K_in);
    hipLaunchKernelGGL(k_mask_noise, grid, dim3(256), 0, st, e1, e2, E, K_in, n_rows, L, N, lc);
    return hipGetLastError();
}

hipError_t launch_mask_combine(const uint32_t *S, const uint32_t *bhat, uint32_t *E, uint32_t K_in, uint32_t n_rows,
                               uint32_t L, uint32_t N, const LimbConsts &lc, hipStream_t st) {
    dim3 grid((N + 255) / 256, n_rows * L * 2 * K_in);
    hipLaunchKernelGGL(k_mask_combine, grid, dim3(256), 0, st, S, bhat, E, K_in, L, N, lc);
    return hipGetLastError();
}
