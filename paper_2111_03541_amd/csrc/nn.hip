// Learned preconditioner for PCG on structured-grid systems: a small linear multilevel
// 3D convolution network, with inference and training kernels written here.  BF16
// storage for weights and activations, FP32 accumulation, FP64 at the PCG boundary.
//
//   z = Dm^-1/2 * N(v),   v = Dm^-1/2 r,   Dm = diag(K)   (BF16 has the exponent range of
//   FP32 and N is linear, so the residual needs no rescaling)
//   N(v) = y_0 + P(y_1 + P(y_2 + ... ))
//   y_0 = conv(v)  (1 -> 1);   y_l = conv(conv(conv(R^l v)))  (1 -> c_l -> c_l -> 1)
//   R: full weighting from a (2n-1)-node grid to an n-node grid; P = R^T (trilinear).
//   3x3x3 convolutions, zero padding, no bias (N is linear in v).  z = 0 on Dirichlet rows.
// Training loss for a residual r: |K z - r|^2 / |r|^2, minimised by Adam; the gradient
// is the adjoint of the linear network (weight gradients only, v does not depend on the
// parameters).  Convolutions have at most 8 channels here, so they are bandwidth- and
// latency-bound and run on the vector units; no MFMA is used in this file.  Inference
// fuses the three convolutions and the prolongation of each level into one kernel over
// LDS tiles; training keeps them separate because the weight gradients need h1 and h2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "mf_internal.h"
#include "pcg.h"

namespace mf {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxLevels = 6;
constexpr int kMaxC = 8;
constexpr int kChunk = 8192;  // points per wgrad block

typedef uint16_t bf16;

__device__ __forceinline__ float bf2f(bf16 v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ bf16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (bf16)(u >> 16);
}
template <typename T>
__device__ __forceinline__ float ld(const T* p, int64_t i);
template <>
__device__ __forceinline__ float ld<bf16>(const bf16* p, int64_t i) { return bf2f(p[i]); }
template <>
__device__ __forceinline__ float ld<float>(const float* p, int64_t i) { return p[i]; }
template <typename T>
__device__ __forceinline__ void st(T* p, int64_t i, float v);
template <>
__device__ __forceinline__ void st<bf16>(bf16* p, int64_t i, float v) { p[i] = f2bf(v); }
template <>
__device__ __forceinline__ void st<float>(float* p, int64_t i, float v) { p[i] = v; }

struct Grid {
    int nx, ny, nz;
    __host__ __device__ int64_t n() const { return (int64_t)nx * ny * nz; }
};

// ---------------- transfer operators ----------------

// coarse(i,j,k) = sum over d in {-1,0,1}^3 of prod 0.5^|d| * fine(2i+dx, 2j+dy, 2k+dz)
template <typename TI, typename TO>
__global__ void k_restrict(const TI* __restrict__ f, Grid gf, TO* __restrict__ c, Grid gc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= gc.n()) return;
    const int i = (int)(t % gc.nx), j = (int)((t / gc.nx) % gc.ny), k = (int)(t / ((int64_t)gc.nx * gc.ny));
    float s = 0.f;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        const int z = 2 * k + dz;
        if (z < 0 || z >= gf.nz) continue;
        const float wz = dz ? 0.5f : 1.f;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = 2 * j + dy;
            if (y < 0 || y >= gf.ny) continue;
            const float wy = wz * (dy ? 0.5f : 1.f);
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = 2 * i + dx;
                if (x < 0 || x >= gf.nx) continue;
                s += wy * (dx ? 0.5f : 1.f) * ld(f, x + (int64_t)gf.nx * (y + (int64_t)gf.ny * z));
            }
        }
    }
    st(c, t, s);
}

// out(fine) = y(fine) + (P c)(fine), trilinear interpolation from the coarse grid
__global__ void k_prolong_add(const float* __restrict__ c, Grid gc, const float* __restrict__ y, float* __restrict__ out,
                              Grid gf)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= gf.n()) return;
    const int x = (int)(t % gf.nx), yy = (int)((t / gf.nx) % gf.ny), z = (int)(t / ((int64_t)gf.nx * gf.ny));
    const int x0 = x >> 1, x1 = (x + 1) >> 1, y0 = yy >> 1, y1 = (yy + 1) >> 1, z0 = z >> 1, z1 = (z + 1) >> 1;
    auto C = [&](int a, int b, int d) { return c[a + (int64_t)gc.nx * (b + (int64_t)gc.ny * d)]; };
    const float v = 0.125f * (C(x0, y0, z0) + C(x1, y0, z0) + C(x0, y1, z0) + C(x1, y1, z0) + C(x0, y0, z1) +
                              C(x1, y0, z1) + C(x0, y1, z1) + C(x1, y1, z1));
    out[t] = (y ? y[t] : 0.f) + v;
}

// ---------------- convolution ----------------

// out[co][p] = sum_ci sum_t w[co][ci][t] in[ci][p + d_t]   (forward)
// dgrad: out[ci][p] = sum_co sum_t w[co][ci][t] in[co][p - d_t]  (transpose = true)
// Weights are FP32 copies of the BF16-rounded parameters.
template <int CIN, int COUT, bool TRANS, typename TI, typename TO>
__global__ void __launch_bounds__(kThreads) k_conv(const TI* __restrict__ in, const float* __restrict__ w,
                                                   TO* __restrict__ out, Grid g)
{
    const int64_t n = g.n();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % g.nx), y = (int)((t / g.nx) % g.ny), z = (int)(t / ((int64_t)g.nx * g.ny));
    float acc[COUT];
#pragma unroll
    for (int o = 0; o < COUT; ++o) acc[o] = 0.f;
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) {
        const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
        const int sx = TRANS ? x - dx : x + dx, sy = TRANS ? y - dy : y + dy, sz = TRANS ? z - dz : z + dz;
        if (sx < 0 || sx >= g.nx || sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz) continue;
        const int64_t q = sx + (int64_t)g.nx * (sy + (int64_t)g.ny * sz);
#pragma unroll
        for (int i = 0; i < CIN; ++i) {
            const float xv = ld(in, (int64_t)i * n + q);
#pragma unroll
            for (int o = 0; o < COUT; ++o) {
                // forward weight index [o][i][tap]; transpose: input channel i is the
                // forward output channel, output channel o the forward input channel
                const float wv = TRANS ? w[(i * COUT + o) * 27 + tap] : w[(o * CIN + i) * 27 + tap];
                acc[o] = fmaf(wv, xv, acc[o]);
            }
        }
    }
#pragma unroll
    for (int o = 0; o < COUT; ++o) st(out, (int64_t)o * n + t, acc[o]);
}

// Inference for one level l >= 1, fused over a T^3 tile of output points: the input v_l
// with a three-point halo, h1 = conv_1(v) and h2 = conv_2(h1) on the shrinking halos (BF16
// in LDS, zero outside the grid, as the unfused kernels store them), y = conv_3(h2), and
// out = y + P coarse (coarse == nullptr on the coarsest level).  The arithmetic order per
// point is that of k_conv and k_prolong_add.
template <int C, int T>
struct LevelSmem {
    static constexpr int A = T + 6, B = T + 4, D = T + 2;  // tile edges of v, h1, h2
    float sv[A * A * A];
    // channel-minor, so that the C channels of one point are one 8- or 16-byte read
    bf16 sh1[B * B * B][C];
    bf16 sh2[D * D * D][C];
    // The weights are not staged: every weight index below is uniform across the wave,
    // so they are scalar loads (SGPR operands of the FMAs) and cost no LDS issue slots.
};

template <int C, int T>
__device__ __forceinline__ void level_tile(const bf16* __restrict__ v, Grid g, const float* __restrict__ w1,
                                           const float* __restrict__ w2, const float* __restrict__ w3,
                                           const float* __restrict__ coarse, Grid gc, float* __restrict__ out,
                                           int bt, LevelSmem<C, T>& S)
{
    constexpr int A = T + 6, B = T + 4, D = T + 2;
    float* sv = S.sv;
    auto& sh1 = S.sh1;
    auto& sh2 = S.sh2;
    const int tid = threadIdx.x;
    const int ntx = (g.nx + T - 1) / T, nty = (g.ny + T - 1) / T;
    const int x0 = (bt % ntx) * T, y0 = ((bt / ntx) % nty) * T, z0 = (bt / (ntx * nty)) * T;
    auto inside = [&](int x, int y, int z) {
        return x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
    };
    for (int i = tid; i < A * A * A; i += kThreads) {
        const int lx = i % A, ly = (i / A) % A, lz = i / (A * A);
        const int x = x0 - 3 + lx, y = y0 - 3 + ly, z = z0 - 3 + lz;
        sv[i] = inside(x, y, z) ? bf2f(v[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)]) : 0.f;
    }
    __syncthreads();
    for (int i = tid; i < B * B * B; i += kThreads) {
        const int lx = i % B, ly = (i / B) % B, lz = i / (B * B);
        float a[C];
#pragma unroll
        for (int o = 0; o < C; ++o) a[o] = 0.f;
        if (inside(x0 - 2 + lx, y0 - 2 + ly, z0 - 2 + lz)) {
#pragma unroll
            for (int tap = 0; tap < 27; ++tap) {
                const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
                const float xv = sv[(lx + 1 + dx) + A * ((ly + 1 + dy) + A * (lz + 1 + dz))];
#pragma unroll
                for (int o = 0; o < C; ++o) a[o] = fmaf(w1[o * 27 + tap], xv, a[o]);
            }
        }
#pragma unroll
        for (int o = 0; o < C; ++o) sh1[i][o] = f2bf(a[o]);
    }
    __syncthreads();
    for (int i = tid; i < D * D * D; i += kThreads) {
        const int lx = i % D, ly = (i / D) % D, lz = i / (D * D);
        float a[C];
#pragma unroll
        for (int o = 0; o < C; ++o) a[o] = 0.f;
        if (inside(x0 - 1 + lx, y0 - 1 + ly, z0 - 1 + lz)) {
#pragma unroll 1
            for (int tap = 0; tap < 27; ++tap) {
                const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
                const int q = (lx + 1 + dx) + B * ((ly + 1 + dy) + B * (lz + 1 + dz));
#pragma unroll
                for (int ci = 0; ci < C; ++ci) {
                    const float xv = bf2f(sh1[q][ci]);
#pragma unroll
                    for (int o = 0; o < C; ++o) a[o] = fmaf(w2[(o * C + ci) * 27 + tap], xv, a[o]);
                }
            }
        }
#pragma unroll
        for (int o = 0; o < C; ++o) sh2[i][o] = f2bf(a[o]);
    }
    __syncthreads();
    for (int i = tid; i < T * T * T; i += kThreads) {
        const int lx = i % T, ly = (i / T) % T, lz = i / (T * T);
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (!inside(x, y, z)) continue;
        float a = 0.f;
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
            const int q = (lx + 1 + dx) + D * ((ly + 1 + dy) + D * (lz + 1 + dz));
#pragma unroll
            for (int ci = 0; ci < C; ++ci) a = fmaf(w3[ci * 27 + tap], bf2f(sh2[q][ci]), a);
        }
        float p = 0.f;
        if (coarse) {
            const int xa = x >> 1, xb = (x + 1) >> 1, ya = y >> 1, yb = (y + 1) >> 1, za = z >> 1, zb = (z + 1) >> 1;
            auto Cv = [&](int aa, int bb, int dd) { return coarse[aa + (int64_t)gc.nx * (bb + (int64_t)gc.ny * dd)]; };
            p = 0.125f * (Cv(xa, ya, za) + Cv(xb, ya, za) + Cv(xa, yb, za) + Cv(xb, yb, za) + Cv(xa, ya, zb) +
                          Cv(xb, ya, zb) + Cv(xa, yb, zb) + Cv(xb, yb, zb));
        }
        out[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)] = a + p;
    }
}


template <int C, int T>
__global__ void __launch_bounds__(kThreads) k_level_fused(const bf16* __restrict__ v, Grid g,
                                                          const float* __restrict__ w1, const float* __restrict__ w2,
                                                          const float* __restrict__ w3,
                                                          const float* __restrict__ coarse, Grid gc,
                                                          float* __restrict__ out)
{
    __shared__ LevelSmem<C, T> S;
    level_tile<C, T>(v, g, w1, w2, w3, coarse, gc, out, blockIdx.x, S);
}

// The convolution chains of several levels in one launch (they are independent; the
// prolongation chain runs after): level 1 with <C1, T1> tiles, the coarser levels with
// <C2, T2> tiles; workgroup b takes tile b of the first level whose tile range holds it.
struct LevelJob {
    const bf16* v;
    Grid g;
    const float* w1;
    const float* w2;
    const float* w3;
    float* out;
    int tiles;
};
struct LevelJobs {
    LevelJob j[kMaxLevels];
    int n;
};

template <int C1, int T1, int C2, int T2>
__global__ void __launch_bounds__(kThreads) k_levels(LevelJobs J)
{
    __shared__ union {
        LevelSmem<C1, T1> a;
        LevelSmem<C2, T2> b;
    } U;
    int b = blockIdx.x, l = 0;
    while (l < J.n - 1 && b >= J.j[l].tiles) {
        b -= J.j[l].tiles;
        ++l;
    }
    const LevelJob& q = J.j[l];
    if (l == 0)
        level_tile<C1, T1>(q.v, q.g, q.w1, q.w2, q.w3, nullptr, q.g, q.out, b, U.a);
    else
        level_tile<C2, T2>(q.v, q.g, q.w1, q.w2, q.w3, nullptr, q.g, q.out, b, U.b);
}

// partial[(o*CIN + i)*27 + tap][chunk] = sum over the chunk of gy[o][p] * x[i][p + d_tap]
template <typename TX>
__global__ void __launch_bounds__(kThreads) k_wgrad(const TX* __restrict__ x, const float* __restrict__ gy, int cin,
                                                    int cout, Grid g, float* __restrict__ partial, int nchunks)
{
    __shared__ float sh[kThreads / 64][27];
    const int pair = blockIdx.y;  // o * cin + i
    const int o = pair / cin, i = pair % cin;
    const int chunk = blockIdx.x;
    const int64_t n = g.n();
    float acc[27];
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) acc[tap] = 0.f;
    const int64_t p0 = (int64_t)chunk * kChunk;
    const int64_t p1 = p0 + kChunk < n ? p0 + kChunk : n;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += kThreads) {
        const float gv = gy[(int64_t)o * n + p];
        const int xx = (int)(p % g.nx), yy = (int)((p / g.nx) % g.ny), zz = (int)(p / ((int64_t)g.nx * g.ny));
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
            const int sx = xx + dx, sy = yy + dy, sz = zz + dz;
            if (sx < 0 || sx >= g.nx || sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz) continue;
            acc[tap] = fmaf(gv, ld(x, (int64_t)i * n + sx + (int64_t)g.nx * (sy + (int64_t)g.ny * sz)), acc[tap]);
        }
    }
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) {
        float v = acc[tap];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (ln == 0) sh[wv][tap] = v;
    }
    __syncthreads();
    if (threadIdx.x < 27) {
        float s = 0.f;
        for (int k = 0; k < kThreads / 64; ++k) s += sh[k][threadIdx.x];
        partial[((int64_t)pair * 27 + threadIdx.x) * nchunks + chunk] = s;
    }
}

// grad[off + j] = sum over chunks of partial[j][chunk]   (fixed order)
__global__ void k_wgrad_reduce(const float* __restrict__ partial, int n_w, int nchunks, float* __restrict__ grad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_w) return;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += partial[(int64_t)j * nchunks + c];
    grad[j] = s;
}

// ---------------- scaling, loss, optimiser ----------------

__global__ void k_diag_scale(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const double* __restrict__ v, int64_t n, const uint8_t* __restrict__ mask,
                             float* __restrict__ dm, uint8_t* __restrict__ m_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) d = v[k];
    dm[i] = d > 0.0 ? (float)(1.0 / sqrt(d)) : 0.f;
    m_out[i] = mask ? mask[i] : 0;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void k_input(const double* __restrict__ r, const float* __restrict__ dm, int64_t n, bf16* __restrict__ v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = f2bf((float)r[i] * dm[i]);
}

// z = Dm^-1/2 (conv_0(v0) + P acc_1), 0 on Dirichlet rows: the level-0 convolution, the
// last prolongation and the output scaling in one pass.  acc1 == nullptr for one level.
// Also stores the level-0 output sum in y0 when y0 != nullptr (training).
__global__ void __launch_bounds__(kThreads) k_final(const bf16* __restrict__ v0, const float* __restrict__ w0,
                                                    const float* __restrict__ acc1, Grid gc, Grid g,
                                                    const float* __restrict__ dm, const uint8_t* __restrict__ mask,
                                                    double* __restrict__ z, float* __restrict__ y0)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.n()) return;
    const int x = (int)(t % g.nx), y = (int)((t / g.nx) % g.ny), zz = (int)(t / ((int64_t)g.nx * g.ny));
    float acc = 0.f;
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) {
        const int sx = x + tap % 3 - 1, sy = y + (tap / 3) % 3 - 1, sz = zz + tap / 9 - 1;
        if (sx < 0 || sx >= g.nx || sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz) continue;
        acc = fmaf(w0[tap], bf2f(v0[sx + (int64_t)g.nx * (sy + (int64_t)g.ny * sz)]), acc);
    }
    if (acc1) {
        const int x0 = x >> 1, x1 = (x + 1) >> 1, y0i = y >> 1, y1 = (y + 1) >> 1, z0 = zz >> 1, z1 = (zz + 1) >> 1;
        auto C = [&](int a, int b, int d) { return acc1[a + (int64_t)gc.nx * (b + (int64_t)gc.ny * d)]; };
        acc += 0.125f * (C(x0, y0i, z0) + C(x1, y0i, z0) + C(x0, y1, z0) + C(x1, y1, z0) + C(x0, y0i, z1) +
                         C(x1, y0i, z1) + C(x0, y1, z1) + C(x1, y1, z1));
    }
    if (y0) y0[t] = acc;
    z[t] = mask[t] ? 0.0 : (double)dm[t] * (double)acc;
}

// v0 = bf16(Dm^-1/2 r) on the fine grid (threads [0, n0)) and v1 = R v0 on the first coarse
// grid (threads [n0, n0 + n1)), v1 recomputing the rounded v0 values it needs; the same
// arithmetic as k_input followed by k_restrict.
__global__ void __launch_bounds__(kThreads) k_input_restrict(const double* __restrict__ r,
                                                             const float* __restrict__ dm, Grid gf,
                                                             bf16* __restrict__ v0, Grid gc, bf16* __restrict__ v1)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n0 = gf.n();
    if (t < n0) {
        v0[t] = f2bf((float)r[t] * dm[t]);
        return;
    }
    const int64_t c = t - n0;
    if (c >= gc.n()) return;
    const int i = (int)(c % gc.nx), j = (int)((c / gc.nx) % gc.ny), k = (int)(c / ((int64_t)gc.nx * gc.ny));
    float s = 0.f;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        const int z = 2 * k + dz;
        if (z < 0 || z >= gf.nz) continue;
        const float wz = dz ? 0.5f : 1.f;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = 2 * j + dy;
            if (y < 0 || y >= gf.ny) continue;
            const float wy = wz * (dy ? 0.5f : 1.f);
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = 2 * i + dx;
                if (x < 0 || x >= gf.nx) continue;
                const int64_t f = x + (int64_t)gf.nx * (y + (int64_t)gf.ny * z);
                s += wy * (dx ? 0.5f : 1.f) * bf2f(f2bf((float)r[f] * dm[f]));
            }
        }
    }
    v1[c] = f2bf(s);
}

// Inference form of k_final over 8^3 tiles: the level-0 input with a one-point halo and
// the 5^3 coarse values the tile interpolates from are staged in LDS first; same
// arithmetic order per point as k_final.
__global__ void __launch_bounds__(kThreads) k_final_tiled(const bf16* __restrict__ v0, const float* __restrict__ w0,
                                                          const float* __restrict__ acc1, Grid gc, Grid g,
                                                          const float* __restrict__ dm,
                                                          const uint8_t* __restrict__ mask, double* __restrict__ z)
{
    constexpr int T = 8, A = T + 2, CT = T / 2 + 1;
    __shared__ float sv[A * A * A];
    __shared__ float sc[CT * CT * CT];
    const int tid = threadIdx.x;
    const int ntx = (g.nx + T - 1) / T, nty = (g.ny + T - 1) / T;
    const int bt = blockIdx.x;
    const int x0 = (bt % ntx) * T, y0 = ((bt / ntx) % nty) * T, z0 = (bt / (ntx * nty)) * T;
    for (int i = tid; i < A * A * A; i += kThreads) {
        const int x = x0 - 1 + i % A, y = y0 - 1 + (i / A) % A, zz = z0 - 1 + i / (A * A);
        const bool in = x >= 0 && x < g.nx && y >= 0 && y < g.ny && zz >= 0 && zz < g.nz;
        sv[i] = in ? bf2f(v0[x + (int64_t)g.nx * (y + (int64_t)g.ny * zz)]) : 0.f;
    }
    if (acc1) {
        for (int i = tid; i < CT * CT * CT; i += kThreads) {
            const int cx = x0 / 2 + i % CT, cy = y0 / 2 + (i / CT) % CT, cz = z0 / 2 + i / (CT * CT);
            const bool in = cx < gc.nx && cy < gc.ny && cz < gc.nz;
            sc[i] = in ? acc1[cx + (int64_t)gc.nx * (cy + (int64_t)gc.ny * cz)] : 0.f;
        }
    }
    __syncthreads();
    for (int i = tid; i < T * T * T; i += kThreads) {
        const int lx = i % T, ly = (i / T) % T, lz = i / (T * T);
        const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
        if (x >= g.nx || y >= g.ny || zz >= g.nz) continue;
        float acc = 0.f;
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            const int sx = x + tap % 3 - 1, sy = y + (tap / 3) % 3 - 1, sz = zz + tap / 9 - 1;
            if (sx < 0 || sx >= g.nx || sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz) continue;
            acc = fmaf(w0[tap], sv[(lx + tap % 3) + A * ((ly + (tap / 3) % 3) + A * (lz + tap / 9))], acc);
        }
        if (acc1) {
            // coarse corners relative to the tile's first coarse point
            const int ax = (x >> 1) - x0 / 2, bx = ((x + 1) >> 1) - x0 / 2;
            const int ay = (y >> 1) - y0 / 2, by = ((y + 1) >> 1) - y0 / 2;
            const int az = (zz >> 1) - z0 / 2, bz = ((zz + 1) >> 1) - z0 / 2;
            auto C = [&](int a, int b, int d) { return sc[a + CT * (b + CT * d)]; };
            acc += 0.125f * (C(ax, ay, az) + C(bx, ay, az) + C(ax, by, az) + C(bx, by, az) + C(ax, ay, bz) +
                             C(bx, ay, bz) + C(ax, by, bz) + C(bx, by, bz));
        }
        const int64_t t = x + (int64_t)g.nx * (y + (int64_t)g.ny * zz);
        z[t] = mask[t] ? 0.0 : (double)dm[t] * (double)acc;
    }
}

// y = K x (FP64 CSR, one row per thread); partial sums of |y - r|^2 and |r|^2
__global__ void k_residual(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, int64_t n, const double* __restrict__ x,
                           const double* __restrict__ r, double* __restrict__ res, double* __restrict__ partial)
{
    __shared__ double sh[2][kThreads / 64];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) s = fma(v[k], x[ci[k]], s);
        const double e = s - r[i];
        res[i] = e;
        a = fma(e, e, a);
        b = fma(r[i], r[i], b);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x % 64 == 0) {
        sh[0][threadIdx.x / 64] = a;
        sh[1][threadIdx.x / 64] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0;
        for (int k = 0; k < kThreads / 64; ++k) {
            s0 += sh[0][k];
            s1 += sh[1][k];
        }
        partial[2 * blockIdx.x] = s0;
        partial[2 * blockIdx.x + 1] = s1;
    }
}

// energy loss pieces: res = K z - r; partial sums of res.(z - e) and r.e
__global__ void k_residual_energy(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const double* __restrict__ v, int64_t n, const double* __restrict__ z,
                                  const double* __restrict__ r, const double* __restrict__ e,
                                  double* __restrict__ res, double* __restrict__ partial)
{
    __shared__ double sh[2][kThreads / 64];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) s = fma(v[k], z[ci[k]], s);
        const double q = s - r[i];
        res[i] = q;
        a = fma(q, z[i] - e[i], a);
        b = fma(r[i], e[i], b);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x % 64 == 0) {
        sh[0][threadIdx.x / 64] = a;
        sh[1][threadIdx.x / 64] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0;
        for (int k = 0; k < kThreads / 64; ++k) {
            s0 += sh[0][k];
            s1 += sh[1][k];
        }
        partial[2 * blockIdx.x] = s0;
        partial[2 * blockIdx.x + 1] = s1;
    }
}

// energy loss gradient: dL/dz = 2 (K z - r) / (r.e), scaled into the network output
__global__ void k_out_grad_energy(const double* __restrict__ res, int64_t n, const double* __restrict__ sums,
                                  const float* __restrict__ dm, const uint8_t* __restrict__ mask,
                                  float* __restrict__ g)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gz = mask[i] ? 0.0 : 2.0 * res[i] / sums[1];
    g[i] = (float)((double)dm[i] * gz);
}

__global__ void k_loss_final(const double* __restrict__ partial, int nb, double* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0, b = 0;
    for (int k = 0; k < nb; ++k) {
        a += partial[2 * k];
        b += partial[2 * k + 1];
    }
    out[0] = a;
    out[1] = b;
    out[2] = b > 0 ? a / b : 0.0;
}

// gacc = s * dm * (2 K res / |r|^2), zero on Dirichlet rows (K symmetric)
__global__ void k_out_grad(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, int64_t n, const double* __restrict__ res,
                           const double* __restrict__ sums, const float* __restrict__ dm,
                           const uint8_t* __restrict__ mask, float* __restrict__ g)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) t = fma(v[k], res[ci[k]], t);
    const double gz = mask[i] ? 0.0 : 2.0 * t / sums[1];
    g[i] = (float)((double)dm[i] * gz);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ vv,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    m[i] = b1 * m[i] + (1.f - b1) * gi;
    vv[i] = b2 * vv[i] + (1.f - b2) * gi * gi;
    p[i] -= lr * (m[i] / c1) / (sqrtf(vv[i] / c2) + eps);
}

// BF16-rounded FP32 copy of the parameters used by the forward pass
__global__ void k_round_bf16(const float* __restrict__ p, float* __restrict__ q, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = bf2f(f2bf(p[i]));
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace
}  // namespace mf

// ------------------------------------------------------------------------------------
// Host object
// ------------------------------------------------------------------------------------
struct mf_nn_s {
    int L = 0;
    int ch[mf::kMaxLevels] = {0};
    mf::Grid g[mf::kMaxLevels];
    int64_t n0 = 0;
    int n_params = 0;
    int w_off[3 * mf::kMaxLevels + 1] = {0};  // parameter offsets of conv tensors
    float* p = nullptr;      // master FP32
    float* pb = nullptr;     // BF16-rounded FP32 copy
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    int step = 0;
    uint64_t seed = 0;  // of the initial weights (recorded in checkpoints)
    // activations
    mf::bf16* vin[mf::kMaxLevels] = {nullptr};
    mf::bf16* h1[mf::kMaxLevels] = {nullptr};
    mf::bf16* h2[mf::kMaxLevels] = {nullptr};
    float* y[mf::kMaxLevels] = {nullptr};
    float* acc[mf::kMaxLevels] = {nullptr};
    float* gy[mf::kMaxLevels] = {nullptr};
    float* g1[mf::kMaxLevels] = {nullptr};
    float* g2[mf::kMaxLevels] = {nullptr};
    float* wpart = nullptr;
    int64_t wpart_n = 0;
    // system binding
    const int32_t* rp = nullptr;
    const int32_t* ci = nullptr;
    const double* kv = nullptr;
    float* dm = nullptr;
    uint8_t* mask = nullptr;
    double* zbuf = nullptr;
    double* res = nullptr;
    double* lpart = nullptr;
    double* sums = nullptr;
    std::vector<void*> allocs;
};

namespace {

using namespace mf;

template <typename T>
mf_status nn_alloc(mf_nn_s* N, T** p, int64_t n)
{
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * (size_t)(n > 0 ? n : 1)) != hipSuccess)
        return set_error(MF_ERR_OOM, "learned preconditioner: device allocation failed");
    N->allocs.push_back(q);
    *p = (T*)q;
    return MF_OK;
}

#define NN_TRY(x)                     \
    do {                              \
        mf_status st_ = (x);          \
        if (st_ != MF_OK) return st_; \
    } while (0)

template <bool TRANS, typename TI, typename TO>
mf_status conv_dispatch(int cin, int cout, const TI* in, const float* w, TO* out, Grid g, hipStream_t s)
{
#define MF_CONV(CI, CO)                                                                         \
    if (cin == CI && cout == CO) {                                                              \
        k_conv<CI, CO, TRANS, TI, TO><<<nblk(g.n()), kThreads, 0, s>>>(in, w, out, g);          \
        return MF_OK;                                                                           \
    }
    MF_CONV(1, 1)
    MF_CONV(1, 2) MF_CONV(2, 2) MF_CONV(2, 1)
    MF_CONV(1, 4) MF_CONV(4, 4) MF_CONV(4, 1)
    MF_CONV(1, 8) MF_CONV(8, 8) MF_CONV(8, 1)
#undef MF_CONV
    return set_error(MF_ERR_UNSUPPORTED, "conv %d -> %d channels not instantiated", cin, cout);
}

// forward pass: z (FP64) from r; y0 != nullptr keeps the level-0 output (training)
mf_status nn_forward(mf_nn_s* N, const double* r, double* z, float* y0, hipStream_t s)
{
    const int64_t n = N->n0;
    k_input<<<nblk(n), kThreads, 0, s>>>(r, N->dm, n, N->vin[0]);
    for (int l = 1; l < N->L; ++l)
        k_restrict<bf16, bf16><<<nblk(N->g[l].n()), kThreads, 0, s>>>(N->vin[l - 1], N->g[l - 1], N->vin[l], N->g[l]);
    for (int l = 1; l < N->L; ++l) {
        const int c = N->ch[l];
        const int b = 1 + 3 * (l - 1);
        NN_TRY((conv_dispatch<false, bf16, bf16>(1, c, N->vin[l], N->pb + N->w_off[b], N->h1[l], N->g[l], s)));
        NN_TRY((conv_dispatch<false, bf16, bf16>(c, c, N->h1[l], N->pb + N->w_off[b + 1], N->h2[l], N->g[l], s)));
        NN_TRY((conv_dispatch<false, bf16, float>(c, 1, N->h2[l], N->pb + N->w_off[b + 2], N->y[l], N->g[l], s)));
    }
    // acc_{L-1} = y_{L-1}; acc_l = y_l + P acc_{l+1} for l >= 1; level 0 fused in k_final
    for (int l = N->L - 2; l >= 1; --l) {
        const float* coarse = (l == N->L - 2) ? N->y[l + 1] : N->acc[l + 1];
        k_prolong_add<<<nblk(N->g[l].n()), kThreads, 0, s>>>(coarse, N->g[l + 1], N->y[l], N->acc[l], N->g[l]);
    }
    const float* acc1 = N->L > 2 ? N->acc[1] : (N->L == 2 ? N->y[1] : nullptr);
    k_final<<<nblk(n), kThreads, 0, s>>>(N->vin[0], N->pb + N->w_off[0], acc1, N->L > 1 ? N->g[1] : N->g[0], N->g[0],
                                         N->dm, N->mask, z, y0);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <int T>
mf_status level_fused_dispatch(int c, const bf16* v, Grid g, const float* w1, const float* w2, const float* w3,
                               const float* coarse, Grid gc, float* out, hipStream_t s)
{
    const int64_t tiles = (int64_t)((g.nx + T - 1) / T) * ((g.ny + T - 1) / T) * ((g.nz + T - 1) / T);
#define MF_LEVEL(CC)                                                                                        \
    if (c == CC) {                                                                                          \
        k_level_fused<CC, T><<<(unsigned)tiles, kThreads, 0, s>>>(v, g, w1, w2, w3, coarse, gc, out);     \
        return MF_OK;                                                                                       \
    }
    MF_LEVEL(1) MF_LEVEL(2) MF_LEVEL(4) MF_LEVEL(8)
#undef MF_LEVEL
    return set_error(MF_ERR_UNSUPPORTED, "fused level with %d channels not instantiated", c);
}

// Inference.  For the shipped shape (level 1 with 4 channels on 8^3 tiles, coarser levels
// with 8 channels on 4^3 tiles): the fine input and first restriction in one kernel, the
// other restrictions, the convolution chains of all levels in one launch (they are
// independent), then the prolongation chain acc_l = y_l + P acc_{l+1} and the level-0
// pass.  Any other shape runs one fused kernel per level from the coarsest up, each
// adding the prolongation of the level below it.
mf_status nn_infer(mf_nn_s* N, const double* r, double* z, hipStream_t s)
{
    const int64_t n = N->n0;
    const int L = N->L;
    bool fast = L >= 3 && N->ch[1] == 4 && N->g[1].n() > 50000;
    for (int l = 2; l < L; ++l) fast = fast && N->ch[l] == 8 && N->g[l].n() <= 50000;
    if (fast) {
        k_input_restrict<<<nblk(n + N->g[1].n()), kThreads, 0, s>>>(r, N->dm, N->g[0], N->vin[0], N->g[1],
                                                                     N->vin[1]);
        for (int l = 2; l < L; ++l)
            k_restrict<bf16, bf16><<<nblk(N->g[l].n()), kThreads, 0, s>>>(N->vin[l - 1], N->g[l - 1], N->vin[l],
                                                                         N->g[l]);
        LevelJobs J{};
        int total = 0;
        for (int l = 1; l < L; ++l) {
            const int T = l == 1 ? 8 : 4;
            const Grid g = N->g[l];
            const int b = 1 + 3 * (l - 1);
            LevelJob& q = J.j[l - 1];
            q.v = N->vin[l];
            q.g = g;
            q.w1 = N->pb + N->w_off[b];
            q.w2 = N->pb + N->w_off[b + 1];
            q.w3 = N->pb + N->w_off[b + 2];
            q.out = N->y[l];
            q.tiles = ((g.nx + T - 1) / T) * ((g.ny + T - 1) / T) * ((g.nz + T - 1) / T);
            total += q.tiles;
        }
        J.n = L - 1;
        k_levels<4, 8, 8, 4><<<(unsigned)total, kThreads, 0, s>>>(J);
        for (int l = L - 2; l >= 1; --l) {
            const float* coarse = (l == L - 2) ? N->y[l + 1] : N->acc[l + 1];
            k_prolong_add<<<nblk(N->g[l].n()), kThreads, 0, s>>>(coarse, N->g[l + 1], N->y[l], N->acc[l], N->g[l]);
        }
    } else {
        k_input<<<nblk(n), kThreads, 0, s>>>(r, N->dm, n, N->vin[0]);
        for (int l = 1; l < L; ++l)
            k_restrict<bf16, bf16><<<nblk(N->g[l].n()), kThreads, 0, s>>>(N->vin[l - 1], N->g[l - 1], N->vin[l],
                                                                         N->g[l]);
        for (int l = L - 1; l >= 1; --l) {
            const int b = 1 + 3 * (l - 1);
            const float* coarse = l == L - 1 ? nullptr : (l + 1 == L - 1 ? N->y[l + 1] : N->acc[l + 1]);
            float* out = l == L - 1 ? N->y[l] : N->acc[l];
            const Grid gc = l + 1 < L ? N->g[l + 1] : N->g[l];
            const float* w1 = N->pb + N->w_off[b];
            const float* w2 = N->pb + N->w_off[b + 1];
            const float* w3 = N->pb + N->w_off[b + 2];
            if (N->g[l].n() > 50000)
                NN_TRY(level_fused_dispatch<8>(N->ch[l], N->vin[l], N->g[l], w1, w2, w3, coarse, gc, out, s));
            else
                NN_TRY(level_fused_dispatch<4>(N->ch[l], N->vin[l], N->g[l], w1, w2, w3, coarse, gc, out, s));
        }
    }
    const float* acc1 = L > 2 ? N->acc[1] : (L == 2 ? N->y[1] : nullptr);
    const Grid g0 = N->g[0];
    const unsigned tiles = (unsigned)(((g0.nx + 7) / 8) * ((g0.ny + 7) / 8) * ((g0.nz + 7) / 8));
    k_final_tiled<<<tiles, kThreads, 0, s>>>(N->vin[0], N->pb + N->w_off[0], acc1, L > 1 ? N->g[1] : N->g[0],
                                             g0, N->dm, N->mask, z);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

mf_status nn_apply_cb(void* ctx, const double* r, double* z, hipStream_t s)
{
    return nn_infer((mf_nn_s*)ctx, r, z, s);
}

// weight gradient of conv(x) -> gy into grad[off ...]
template <typename TX>
mf_status wgrad(mf_nn_s* N, const TX* x, const float* gy, int cin, int cout, Grid g, int off, hipStream_t s)
{
    const int nchunks = (int)((g.n() + kChunk - 1) / kChunk);
    const int64_t need = (int64_t)cin * cout * 27 * nchunks;
    if (need > N->wpart_n) return set_error(MF_ERR_ARG, "wgrad scratch too small");
    k_wgrad<TX><<<dim3(nchunks, cin * cout), kThreads, 0, s>>>(x, gy, cin, cout, g, N->wpart, nchunks);
    const int nw = cin * cout * 27;
    k_wgrad_reduce<<<(nw + 255) / 256, 256, 0, s>>>(N->wpart, nw, nchunks, N->grad + off);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

void free_nn(mf_nn_s* N)
{
    if (!N) return;
    for (void* p : N->allocs) (void)hipFree(p);
    delete N;
}

uint64_t splitmix(uint64_t& x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

namespace mf {
mf_status nn_bind_pcg(const mf_nn_t* net, int64_t n_rows, PcgArgs* a)
{
    if (!net->dm || !net->kv) return set_error(MF_ERR_ARG, "call mf_nn_set_system before mf_pcg");
    if (n_rows != net->n0) return set_error(MF_ERR_ARG, "network grid has %lld nodes, system %lld rows",
                                            (long long)net->n0, (long long)n_rows);
    if (a->values != net->kv) return set_error(MF_ERR_ARG, "the network is bound to a different matrix");
    a->precond = MF_PRECOND_EXTERNAL;
    a->apply = nn_apply_cb;
    a->apply_ctx = (void*)net;
    a->apply_graph_safe = 1;
    return MF_OK;
}
}  // namespace mf

extern "C" {

mf_status mf_nn_create(const int32_t* grid, int32_t levels, const int32_t* channels, uint64_t seed, mf_nn_t** out)
{
    if (!out) return set_error(MF_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!grid || !channels) return set_error(MF_ERR_ARG, "grid or channels is NULL");
    if (levels < 1 || levels > kMaxLevels) return set_error(MF_ERR_ARG, "levels must be 1..%d", kMaxLevels);
    if (channels[0] != 1) return set_error(MF_ERR_ARG, "channels[0] must be 1 (the level-0 stencil)");
    mf_nn_s* N = new mf_nn_s();
    N->L = levels;
    N->seed = seed;
    N->g[0] = Grid{grid[0], grid[1], grid[2]};
    for (int l = 0; l < levels; ++l) {
        const int c = channels[l];
        if (l > 0 && !(c == 1 || c == 2 || c == 4 || c == 8)) {
            free_nn(N);
            return set_error(MF_ERR_UNSUPPORTED, "level %d width %d (1, 2, 4 or 8)", l, c);
        }
        N->ch[l] = c;
        if (l > 0) {
            const Grid& f = N->g[l - 1];
            if (f.nx % 2 == 0 || f.ny % 2 == 0 || f.nz % 2 == 0 || f.nx < 3 || f.ny < 3 || f.nz < 3) {
                free_nn(N);
                return set_error(MF_ERR_ARG, "grid %dx%dx%d cannot be coarsened (odd sizes >= 3)", f.nx, f.ny, f.nz);
            }
            N->g[l] = Grid{(f.nx + 1) / 2, (f.ny + 1) / 2, (f.nz + 1) / 2};
        }
    }
    if (N->g[0].nx < 1 || N->g[0].ny < 1 || N->g[0].nz < 1) {
        free_nn(N);
        return set_error(MF_ERR_ARG, "empty grid");
    }
    N->n0 = N->g[0].n();
    // parameter layout: level-0 conv (1x1x27), then per level (c,1) (c,c) (1,c) x 27
    int off = 0, k = 0;
    N->w_off[k++] = off;
    off += 27;
    for (int l = 1; l < levels; ++l) {
        const int c = N->ch[l];
        N->w_off[k++] = off;
        off += c * 27;
        N->w_off[k++] = off;
        off += c * c * 27;
        N->w_off[k++] = off;
        off += c * 27;
    }
    N->n_params = off;
    mf_status st = MF_OK;
    auto A = [&](mf_status x) { if (st == MF_OK) st = x; };
    A(nn_alloc(N, &N->p, off));
    A(nn_alloc(N, &N->pb, off));
    A(nn_alloc(N, &N->grad, off));
    A(nn_alloc(N, &N->m, off));
    A(nn_alloc(N, &N->v, off));
    int64_t wp = 0;
    for (int l = 0; l < levels; ++l) {
        const int64_t n = N->g[l].n();
        const int c = N->ch[l];
        A(nn_alloc(N, &N->vin[l], n));
        A(nn_alloc(N, &N->y[l], n));
        A(nn_alloc(N, &N->acc[l], n));
        A(nn_alloc(N, &N->gy[l], n));
        if (l > 0) {
            A(nn_alloc(N, &N->h1[l], n * c));
            A(nn_alloc(N, &N->h2[l], n * c));
            A(nn_alloc(N, &N->g1[l], n * c));
            A(nn_alloc(N, &N->g2[l], n * c));
        }
        const int64_t chunks = (n + kChunk - 1) / kChunk;
        wp = std::max<int64_t>(wp, (int64_t)std::max(c, 1) * std::max(c, 1) * 27 * chunks);
    }
    N->wpart_n = wp;
    A(nn_alloc(N, &N->wpart, wp));
    A(nn_alloc(N, &N->dm, N->n0));
    A(nn_alloc(N, &N->mask, N->n0));
    A(nn_alloc(N, &N->zbuf, N->n0));
    A(nn_alloc(N, &N->res, N->n0));
    A(nn_alloc(N, &N->lpart, 2 * 1024));
    A(nn_alloc(N, &N->sums, 4));
    if (st != MF_OK) {
        free_nn(N);
        return st;
    }

    // initial parameters: level-0 stencil = identity (the network starts as Jacobi),
    // other weights small Gaussian (splitmix64 + Box-Muller), Adam state zero
    std::vector<float> h(off, 0.f);
    uint64_t x = seed;
    for (int i = 27; i < off; ++i) {
        double u1 = ((splitmix(x) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        double u2 = ((splitmix(x) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        h[i] = (float)(0.02 * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
    h[13] = 1.f;
    std::vector<float> zero(off, 0.f);
    if (hipMemcpy(N->p, h.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(N->m, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(N->v, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess) {
        free_nn(N);
        return set_error(MF_ERR_HIP, "parameter upload failed");
    }
    k_round_bf16<<<(off + 255) / 256, 256>>>(N->p, N->pb, off);
    if (hipDeviceSynchronize() != hipSuccess) {
        free_nn(N);
        return set_error(MF_ERR_HIP, "parameter rounding failed");
    }
    *out = N;
    return MF_OK;
}

mf_status mf_nn_params(mf_nn_t* N, float* get, const float* set, int64_t* n_params)
{
    if (!N) return set_error(MF_ERR_ARG, "network is NULL");
    if (n_params) *n_params = N->n_params;
    if (get) MF_HIP(hipMemcpy(get, N->p, sizeof(float) * N->n_params, hipMemcpyDeviceToHost));
    if (set) {
        MF_HIP(hipMemcpy(N->p, set, sizeof(float) * N->n_params, hipMemcpyHostToDevice));
        std::vector<float> zero(N->n_params, 0.f);
        MF_HIP(hipMemcpy(N->m, zero.data(), sizeof(float) * N->n_params, hipMemcpyHostToDevice));
        MF_HIP(hipMemcpy(N->v, zero.data(), sizeof(float) * N->n_params, hipMemcpyHostToDevice));
        N->step = 0;
        k_round_bf16<<<(N->n_params + 255) / 256, 256>>>(N->p, N->pb, N->n_params);
        MF_HIP(hipDeviceSynchronize());
    }
    return MF_OK;
}

mf_status mf_nn_set_system(mf_nn_t* N, const mf_csr* K, const uint8_t* dirichlet, void* stream)
{
    if (!N || !K) return set_error(MF_ERR_ARG, "network or matrix is NULL");
    if (K->n_rows != N->n0) return set_error(MF_ERR_ARG, "matrix has %lld rows, network grid %lld nodes",
                                             (long long)K->n_rows, (long long)N->n0);
    hipStream_t s = (hipStream_t)stream;
    N->rp = K->row_ptr;
    N->ci = K->col_idx;
    N->kv = K->values;
    k_diag_scale<<<nblk(N->n0), kThreads, 0, s>>>(K->row_ptr, K->col_idx, K->values, N->n0, dirichlet, N->dm, N->mask);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

mf_status mf_nn_apply(mf_nn_t* N, const double* r, double* z, void* stream)
{
    if (!N || !r || !z) return set_error(MF_ERR_ARG, "NULL argument");
    if (!N->kv) return set_error(MF_ERR_ARG, "call mf_nn_set_system first");
    return nn_apply_cb(N, r, z, (hipStream_t)stream);
}

mf_status mf_nn_train_step(mf_nn_t* N, const double* r, const double* e, double lr, double* loss, float* grad_out,
                           void* stream)
{
    if (!N || !r) return set_error(MF_ERR_ARG, "NULL argument");
    if (!N->kv) return set_error(MF_ERR_ARG, "call mf_nn_set_system first");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = N->n0;
    NN_TRY(nn_forward(N, r, N->zbuf, nullptr, s));
    const unsigned nb = (unsigned)std::min<int64_t>(1024, nblk(n));
    if (e) {
        k_residual_energy<<<nb, kThreads, 0, s>>>(N->rp, N->ci, N->kv, n, N->zbuf, r, e, N->res, N->lpart);
        k_loss_final<<<1, 64, 0, s>>>(N->lpart, nb, N->sums);
        k_out_grad_energy<<<nblk(n), kThreads, 0, s>>>(N->res, n, N->sums, N->dm, N->mask, N->gy[0]);
    } else {
        k_residual<<<nb, kThreads, 0, s>>>(N->rp, N->ci, N->kv, n, N->zbuf, r, N->res, N->lpart);
        k_loss_final<<<1, 64, 0, s>>>(N->lpart, nb, N->sums);
        k_out_grad<<<nblk(n), kThreads, 0, s>>>(N->rp, N->ci, N->kv, n, N->res, N->sums, N->dm, N->mask, N->gy[0]);
    }
    for (int l = 1; l < N->L; ++l)
        k_restrict<float, float><<<nblk(N->g[l].n()), kThreads, 0, s>>>(N->gy[l - 1], N->g[l - 1], N->gy[l], N->g[l]);
    NN_TRY(wgrad<bf16>(N, N->vin[0], N->gy[0], 1, 1, N->g[0], N->w_off[0], s));
    for (int l = 1; l < N->L; ++l) {
        const int c = N->ch[l];
        const int b = 1 + 3 * (l - 1);
        NN_TRY(wgrad<bf16>(N, N->h2[l], N->gy[l], c, 1, N->g[l], N->w_off[b + 2], s));
        NN_TRY((conv_dispatch<true, float, float>(1, c, N->gy[l], N->pb + N->w_off[b + 2], N->g2[l], N->g[l], s)));
        NN_TRY(wgrad<bf16>(N, N->h1[l], N->g2[l], c, c, N->g[l], N->w_off[b + 1], s));
        NN_TRY((conv_dispatch<true, float, float>(c, c, N->g2[l], N->pb + N->w_off[b + 1], N->g1[l], N->g[l], s)));
        NN_TRY(wgrad<bf16>(N, N->vin[l], N->g1[l], 1, c, N->g[l], N->w_off[b], s));
    }
    double h[3] = {0, 0, 0};
    MF_HIP(hipMemcpyAsync(h, N->sums, sizeof(h), hipMemcpyDeviceToHost, s));
    if (grad_out) MF_HIP(hipMemcpyAsync(grad_out, N->grad, sizeof(float) * N->n_params, hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    if (loss) *loss = h[2];
    if (!std::isfinite(h[2])) return set_error(MF_ERR_NONFINITE, "non-finite training loss");
    if (!grad_out && lr > 0.0) {
        N->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - std::pow(b1, (float)N->step), c2 = 1.f - std::pow(b2, (float)N->step);
        k_adam<<<(N->n_params + 255) / 256, 256, 0, s>>>(N->p, N->grad, N->m, N->v, N->n_params, (float)lr, b1, b2,
                                                        1e-8f, c1, c2);
        k_round_bf16<<<(N->n_params + 255) / 256, 256, 0, s>>>(N->p, N->pb, N->n_params);
        MF_HIP(hipGetLastError());
    }
    return MF_OK;
}

// Checkpoint layout (host bytes, little endian): header of 16 int64 words
//   [0] magic "MFNNCKP1", [1] n_params, [2] step, [3] seed, [4] levels,
//   [5..7] node grid, [8..8+levels) channels, rest zero;
// then the FP32 parameters, the first Adam moments and the second Adam moments.
namespace {
constexpr int64_t kCkpMagic = 0x31504B434E4E464DLL;  // "MFNNCKP1"
constexpr int kCkpHeader = 16;
int64_t ckp_bytes(const mf_nn_s* N) { return (int64_t)sizeof(int64_t) * kCkpHeader + 3 * (int64_t)sizeof(float) * N->n_params; }
}  // namespace

mf_status mf_nn_checkpoint_size(const mf_nn_t* N, int64_t* bytes)
{
    if (!N || !bytes) return set_error(MF_ERR_ARG, "NULL argument");
    *bytes = ckp_bytes(N);
    return MF_OK;
}

mf_status mf_nn_save(const mf_nn_t* N, void* buf, int64_t bytes)
{
    if (!N || !buf) return set_error(MF_ERR_ARG, "NULL argument");
    if (bytes < ckp_bytes(N)) return set_error(MF_ERR_ARG, "checkpoint buffer of %lld bytes, %lld needed",
                                               (long long)bytes, (long long)ckp_bytes(N));
    int64_t* h = (int64_t*)buf;
    for (int k = 0; k < kCkpHeader; ++k) h[k] = 0;
    h[0] = kCkpMagic;
    h[1] = N->n_params;
    h[2] = N->step;
    h[3] = (int64_t)N->seed;
    h[4] = N->L;
    h[5] = N->g[0].nx;
    h[6] = N->g[0].ny;
    h[7] = N->g[0].nz;
    for (int l = 0; l < N->L; ++l) h[8 + l] = N->ch[l];
    float* f = (float*)(h + kCkpHeader);
    MF_HIP(hipDeviceSynchronize());
    MF_HIP(hipMemcpy(f, N->p, sizeof(float) * N->n_params, hipMemcpyDeviceToHost));
    MF_HIP(hipMemcpy(f + N->n_params, N->m, sizeof(float) * N->n_params, hipMemcpyDeviceToHost));
    MF_HIP(hipMemcpy(f + 2 * (int64_t)N->n_params, N->v, sizeof(float) * N->n_params, hipMemcpyDeviceToHost));
    return MF_OK;
}

mf_status mf_nn_load(mf_nn_t* N, const void* buf, int64_t bytes)
{
    if (!N || !buf) return set_error(MF_ERR_ARG, "NULL argument");
    if (bytes < (int64_t)sizeof(int64_t) * kCkpHeader) return set_error(MF_ERR_ARG, "checkpoint too short");
    const int64_t* h = (const int64_t*)buf;
    if (h[0] != kCkpMagic) return set_error(MF_ERR_ARG, "not a network checkpoint");
    bool same = h[1] == N->n_params && h[4] == N->L && h[5] == N->g[0].nx && h[6] == N->g[0].ny && h[7] == N->g[0].nz;
    for (int l = 0; same && l < N->L; ++l) same = h[8 + l] == N->ch[l];
    if (!same) return set_error(MF_ERR_ARG, "checkpoint of a different network (grid, levels or channels)");
    if (bytes < ckp_bytes(N)) return set_error(MF_ERR_ARG, "checkpoint truncated");
    const float* f = (const float*)(h + kCkpHeader);
    MF_HIP(hipDeviceSynchronize());
    MF_HIP(hipMemcpy(N->p, f, sizeof(float) * N->n_params, hipMemcpyHostToDevice));
    MF_HIP(hipMemcpy(N->m, f + N->n_params, sizeof(float) * N->n_params, hipMemcpyHostToDevice));
    MF_HIP(hipMemcpy(N->v, f + 2 * (int64_t)N->n_params, sizeof(float) * N->n_params, hipMemcpyHostToDevice));
    N->step = (int)h[2];
    N->seed = (uint64_t)h[3];
    k_round_bf16<<<(N->n_params + 255) / 256, 256>>>(N->p, N->pb, N->n_params);
    MF_HIP(hipDeviceSynchronize());
    return MF_OK;
}

void mf_nn_destroy(mf_nn_t* N)
{
    if (!N) return;
    (void)hipDeviceSynchronize();
    free_nn(N);
}

}  // extern "C"
