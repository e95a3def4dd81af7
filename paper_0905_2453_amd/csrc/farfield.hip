// Learned far-field closure on gfx950.
//
// The deflection of a ray (Thompson et al. 2009, section 1 eq. 2) is split per ray tile into
// a near part, summed exactly over the lenses closer than r_near to the tile rectangle, and a
// far part (the rest of the sum, the lens subsets of section 2 eq. 5).  The far part is
// represented per tile by an exact FP64 affine base at the tile centre plus a small network
// fitted to exact far-field sums:
//   alpha_far(x) ~ alpha_far(c) + J_far(c) (x - c) + s_t * net((x - c) / h)
// net: 16 Fourier features -> 64 -> 64 -> 2 (SiLU), bfloat16 GEMM operands, FP32 sums.
//
// Hidden-unit layout.  A 32x32x16 MFMA leaves in lane l (half hf = l / 32, column l % 32) the
// output rows 32 T + 8 (r / 4) + 4 hf + r % 4 of tile T, register r.  The rows of every weight
// matrix that produces hidden units are permuted (perm_row) so that register r of tile T holds
// hidden unit slot_unit(16 T + r, hf): exactly the B-operand layout of the next 32x32x16 MFMA
// over hidden units.  So each lane keeps the 32 hidden values of its sample it needs, and the
// forward pass and the data half of the backward pass need no cross-lane moves.  The weight
// gradients contract over samples and go through small per-wave LDS transposes.
#include <algorithm>

#include "rs_internal.h"

namespace rs {

namespace {

using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using u16x8 = unsigned short __attribute__((ext_vector_type(8)));
using f32x16 = float __attribute__((ext_vector_type(16)));
using f32x4 = float __attribute__((ext_vector_type(4)));

constexpr double kRcpBiasComp = 1.0 + 6.41e-9;  // see direct.hip: mean bias of v_rcp_f32
constexpr float kPadCoord = 1.0e18f;

// float -> bfloat16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

using u32x4 = uint32_t __attribute__((ext_vector_type(4)));
using bf16x2 = __bf16 __attribute__((ext_vector_type(2)));
using f32x2 = float __attribute__((ext_vector_type(2)));

// two floats -> a bfloat16 pair (a in the low half), round to nearest even (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pk2(float a, float b)
{
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float lo_bf16(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float hi_bf16(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

__device__ __forceinline__ bf16x8 lds8(const uint16_t *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(p));
}
// four bfloat16 pairs -> the 8-element MFMA operand (pair j gives elements 2j, 2j + 1)
__device__ __forceinline__ bf16x8 pack4(const uint32_t *p)
{
    const u32x4 v = {p[0], p[1], p[2], p[3]};
    return __builtin_bit_cast(bf16x8, v);
}

// logical hidden unit produced by output row R (0..63) of a hidden-producing layer
__device__ __forceinline__ int perm_row(int R)
{
    const int T = R >> 5, rr = R & 31, a = rr >> 3, hf = (rr >> 2) & 1, b = rr & 3;
    return 32 * T + 16 * (a >> 1) + 8 * hf + 4 * (a & 1) + b;
}
// The 64 x 64 bfloat16 matrices in LDS (W2, and its transpose in training) keep the 16-byte chunk c of
// row r at position c ^ wsw(r): the eight rows that one MFMA operand load reads together (rows
// 8 h + b of a 32-row tile, h < 2, b < 4) then fall on eight different bank groups, and so do the
// column writes of the optimiser update.
__device__ __forceinline__ int wsw(int r) { return (r & 3) | (((r >> 3) & 1) << 2); }
__device__ __forceinline__ int m64(int r, int c) { return r * 64 + ((((c >> 3) ^ wsw(r)) << 3) | (c & 7)); }
// LDS position of parameter p in the flat bfloat16 weight array (W2 swizzled as above)
__device__ __forceinline__ int wslot(int p)
{
    return (p >= kOffW2 && p < kOffB2) ? kOffW2 + m64((p - kOffW2) >> 6, (p - kOffW2) & 63) : p;
}
// logical hidden unit held in slot q (0..31) by a lane of half hf
__device__ __forceinline__ int slot_unit(int q, int hf) { return 16 * (q >> 3) + 8 * hf + (q & 7); }

// sigmoid with the hardware reciprocal (1 ulp): its error is far below the bfloat16 rounding
// every activation and delta goes through
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// Lens (FP32 record) within r_near of the tile rectangle, decided in FP64.
__device__ __forceinline__ bool is_near(float lx, float ly, const double lo[2], const double hi[2], double rn2)
{
    const double x = lx, y = ly;
    const double ex = fmax(fmax(lo[0] - x, x - hi[0]), 0.0);
    const double ey = fmax(fmax(lo[1] - y, y - hi[1]), 0.0);
    return ex * ex + ey * ey < rn2;
}

__device__ __forceinline__ float ray_coord(double lo, double t, int64_t i, double u = 0.5)
{
    double v = ((double)i + u) * t;
    double w = lo + v;
    return (float)w;
}

// Tile rectangle (cells of the tile's rays), centre and half-widths.
__device__ __forceinline__ void tile_geom(const FarArgs &f, uint32_t tile, double lo[2], double hi[2], double c[2],
                                          double hw[2], int64_t i0[2], int n[2])
{
    const int tx = (int)(tile % (uint32_t)f.tiles_x), ty = (int)(tile / (uint32_t)f.tiles_x);
    i0[0] = f.wlo1 + (int64_t)tx * f.TX;
    i0[1] = f.wlo2 + (int64_t)ty * f.TY;
    n[0] = (int)min((int64_t)f.TX, f.wlo1 + f.wn1 - i0[0]);
    n[1] = (int)min((int64_t)f.TY, f.wlo2 + f.wn2 - i0[1]);
    lo[0] = f.glo1 + (double)i0[0] * f.gt1;
    lo[1] = f.glo2 + (double)i0[1] * f.gt2;
    hi[0] = f.glo1 + (double)(i0[0] + n[0]) * f.gt1;
    hi[1] = f.glo2 + (double)(i0[1] + n[1]) * f.gt2;
    c[0] = 0.5 * (lo[0] + hi[0]);
    c[1] = 0.5 * (lo[1] + hi[1]);
    hw[0] = 0.5 * (hi[0] - lo[0]);
    hw[1] = 0.5 * (hi[1] - lo[1]);
}

__device__ __forceinline__ double *tile_hdr(const FarArgs &f, uint32_t tile)
{
    return reinterpret_cast<double *>(f.model + kModelHeader + (size_t)tile * kTileRecord);
}
__device__ __forceinline__ uint16_t *tile_w(const FarArgs &f, uint32_t tile)
{
    return reinterpret_cast<uint16_t *>(f.model + kModelHeader + (size_t)tile * kTileRecord + kTileWeightsOff);
}

// Features of one axis for a lane: phi[8 hf + 2k] = sin(w_k u), phi[8 hf + 2k + 1] = cos(w_k u),
// w_k = (pi / 2) 2^k, rounded to bfloat16 (pair k of out: sine low, cosine high).  w_k u is
// 2 pi (2^(k-2) u), an exact scaling of u, so each value is one hardware sine or cosine of an
// argument in revolutions (|2^(k-2) u| <= 2).
__device__ __forceinline__ void features8(float u, uint32_t *out)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float rev = u * (float)(1 << k) * 0.25f;
        out[k] = pk2(__builtin_amdgcn_sinf(rev), __builtin_amdgcn_cosf(rev));
    }
}

// Forward pass of 32 samples (one per lane pair) through layers 1 and 2: returns the bfloat16
// activations h1, h2 in the slot layout and the network output (both lanes); with TRAIN also
// the SiLU derivatives silu'(z) = s (1 + z (1 - s)) = s + h (1 - s), s = sigmoid(z), h = z s,
// that the backward pass needs.  Activations are kept as bfloat16 pairs: word j holds slot 2j in
// its low half and slot 2j + 1 in its high half, which is the B-operand layout of the next MFMA.
struct Fwd {
    float d1[32], d2[32];
    uint32_t h1[16], h2[16];
    float o[2];
};

// a . b + c over the two bfloat16 halves of a and b, FP32 sum (v_dot2c_f32_bf16)
__device__ __forceinline__ float dot2bf(uint32_t a, uint32_t b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b), c, false);
}

// Layer 3 in training, where the forward pass holds no register to spare: the lane's 32 units of its
// sample as bfloat16 pair dot products (word j of h2 holds slots 2j, 2j + 1, the consecutive units
// 16 g + 8 hf + e, e + 1 with j = 4 g + e / 2, which pair with the consecutive weights of W3's rows),
// two partial sums per output, then the two halves of the sample (lanes l and l ^ 32) in a fixed
// order, plus b3.
__device__ __forceinline__ void layer3_dot(const uint16_t *Wbf, const float *sbias, const uint32_t *h2, int hf,
                                           float &o0, float &o1)
{
    float a[2][2] = {};
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const u32x4 w0 = *reinterpret_cast<const u32x4 *>(Wbf + kOffW3 + 16 * g + 8 * hf);
        const u32x4 w1 = *reinterpret_cast<const u32x4 *>(Wbf + kOffW3 + 64 + 16 * g + 8 * hf);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[g & 1][0] = dot2bf(h2[4 * g + j], w0[j], a[g & 1][0]);
            a[g & 1][1] = dot2bf(h2[4 * g + j], w1[j], a[g & 1][1]);
        }
    }
    const float p0 = a[0][0] + a[1][0], p1 = a[0][1] + a[1][1];
    const float q0 = __shfl_xor(p0, 32), q1 = __shfl_xor(p1, 32);
    o0 = (hf == 0 ? p0 + q0 : q0 + p0) + sbias[128];
    o1 = (hf == 0 ? p1 + q1 : q1 + p1) + sbias[129];
}

// Layer 3 in evaluation (64 units -> 2) of 32 samples as four 32x32x16 MFMAs over the lane's activation pairs (the
// B operand of layer 2's layout): rows 0 and 1 of A are W3's two rows (lanes 0, 1 and 32, 33), the
// other rows read a 16-byte zero block; the accumulator starts at b3.  Output rows 0 and 1 land in
// registers 0 and 1 of the half-0 lanes: o is valid there only (the lanes that use it).
__device__ __forceinline__ void layer3(const uint16_t *Wbf, const float *sbias, const uint16_t *zero16,
                                       const uint32_t *h2, int col, int hf, float &o0, float &o1)
{
    f32x16 acc = {};
    acc[0] = sbias[128];
    acc[1] = sbias[129];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const uint16_t *row = col < 2 ? Wbf + kOffW3 + 64 * col + 16 * kk + 8 * hf : zero16;
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lds8(row), pack4(h2 + 4 * kk), acc, 0, 0, 0);
    }
    o0 = acc[0];
    o1 = acc[1];
}

// The 16 biases of output tile T of a hidden layer, for a lane of half hf, in slot order (units
// 32 T + 8 hf + e and 32 T + 16 + 8 hf + e, e < 8: the order of the MFMA's output registers), as the
// accumulator the tile's first MFMA starts from, so that the matrix unit adds them; four 16-byte
// LDS reads.
__device__ __forceinline__ f32x16 load_bias16(const float *bias, int T, int hf)
{
    const f32x4 *p0 = reinterpret_cast<const f32x4 *>(bias + 32 * T + 8 * hf);
    const f32x4 *p1 = reinterpret_cast<const f32x4 *>(bias + 32 * T + 16 + 8 * hf);
    const f32x4 v0 = p0[0], v1 = p0[1], v2 = p1[0], v3 = p1[1];
    f32x16 b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        b[e] = v0[e];
        b[4 + e] = v1[e];
        b[8 + e] = v2[e];
        b[12 + e] = v3[e];
    }
    return b;
}

// LDS operands are requested before the MFMAs that need them and the activations of the previous
// tile; a scheduling barrier keeps the compiler from sinking the reads next to their use, where
// each would expose its full LDS latency.
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// SiLU of one output tile's pre-activations z (bias included)
template <bool TRAIN>
__device__ __forceinline__ void activate16(const f32x16 &z, int T, float *d, uint32_t *h)
{
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
        const float za = z[q], zb = z[q + 1];
        const float sa = sigm(za), sb = sigm(zb);
        const float ha = za * sa, hb = zb * sb;
        if (TRAIN) {
            d[16 * T + q] = fmaf(ha, 1.0f - sa, sa);
            d[16 * T + q + 1] = fmaf(hb, 1.0f - sb, sb);
        }
        h[(16 * T + q) / 2] = pk2(ha, hb);
    }
}

// Layer 1 (16 features -> 64 units) and layer 2 (64 -> 64) of 32 samples: MFMA (starting from the
// biases), SiLU, with the SiLU derivatives when TRAIN.  Each tile's operands and biases are read
// from LDS before its MFMAs are issued.
template <bool TRAIN>
__device__ __forceinline__ void layer1(const uint16_t *Wbf, const float *sbias, const bf16x8 &bphi, int col, int hf,
                                       float *d1, uint32_t *h1)
{
    bf16x8 a[2];
    f32x16 acc[2];
#pragma unroll
    for (int T = 0; T < 2; ++T) {
        a[T] = lds8(Wbf + kOffW1 + perm_row(32 * T + col) * 16 + 8 * hf);
        acc[T] = load_bias16(sbias, T, hf);
    }
    sched_fence();
#pragma unroll
    for (int T = 0; T < 2; ++T) acc[T] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[T], bphi, acc[T], 0, 0, 0);
#pragma unroll
    for (int T = 0; T < 2; ++T) activate16<TRAIN>(acc[T], T, d1, h1);
}

template <bool TRAIN>
__device__ __forceinline__ void layer2(const uint16_t *Wbf, const float *sbias, const uint32_t *h1, int col, int hf,
                                       float *d2, uint32_t *h2)
{
#pragma unroll
    for (int T = 0; T < 2; ++T) {
        bf16x8 a[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) a[kk] = lds8(Wbf + kOffW2 + m64(perm_row(32 * T + col), 16 * kk + 8 * hf));
        f32x16 acc = load_bias16(sbias + 64, T, hf);
        sched_fence();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kk], pack4(h1 + 4 * kk), acc, 0, 0, 0);
        activate16<TRAIN>(acc, T, d2, h2);
    }
}

template <bool TRAIN>
__device__ __forceinline__ void forward32(const uint16_t *Wbf, const float *sbias, const uint16_t *zero16,
                                          const uint32_t *phi4, int lane, Fwd &r)
{
    const int hf = lane >> 5, col = lane & 31;
    const bf16x8 bphi = pack4(phi4);
    layer1<TRAIN>(Wbf, sbias, bphi, col, hf, r.d1, r.h1);
    layer2<TRAIN>(Wbf, sbias, r.h1, col, hf, r.d2, r.h2);
    layer3(Wbf, sbias, zero16, r.h2, col, hf, r.o[0], r.o[1]);   // valid in the half-0 lanes
}

// ---------------------------------------------------------------- fit: affine base

// alpha_far(c) and its Jacobian over the far set of each tile, FP64; a workgroup takes NT
// consecutive tiles (of the tile list when one is given), so every lens record it loads serves
// all of them (NT = 4 when there are enough tiles to fill the GPU, else 1).  Each tile's sums are those of a workgroup of its own: thread t
// takes lenses t, t + 256, ... in order, then a fixed tree adds the 256 partial sums.  At fit
// time the result goes into the model's tile header.  For a moving field (eval with
// velocities) the far set is still the one chosen by the fit-time positions, each far lens
// enters at its position at f.time, and the result goes to f.affine (only the evaluated tiles).
template <int NT>
__global__ void __launch_bounds__(256) k_ff_affine(const FarArgs f)
{
    constexpr int kAffTiles = NT;
    __shared__ double red[4][256];
    const bool listed = f.affine && f.eval_tiles;
    const int64_t count = listed ? f.n_eval : f.n_tiles;
    const int64_t first = (int64_t)blockIdx.x * kAffTiles;
    const int nt = (int)min((int64_t)kAffTiles, count - first);
    uint32_t tile[kAffTiles];
    double lo[kAffTiles][2], hi[kAffTiles][2], c[kAffTiles][2];
#pragma unroll
    for (int t = 0; t < kAffTiles; ++t) {
        // a short last group repeats its last tile; those sums are never written
        const int64_t e = first + min(t, nt - 1);
        tile[t] = listed ? (uint32_t)f.eval_tiles[e] : (uint32_t)e;
        double hw[2];
        int64_t i0[2];
        int n[2];
        tile_geom(f, tile[t], lo[t], hi[t], c[t], hw, i0, n);
    }
    const double rn2 = f.r_near * f.r_near;
    // the group's bounding box: a lens at least r_near from it is at least r_near from each of
    // its tiles, and the FP64 test is monotone in the box, so skipping the per-tile tests for
    // such a lens decides exactly as they would
    double ulo[2] = {lo[0][0], lo[0][1]}, uhi[2] = {hi[0][0], hi[0][1]};
#pragma unroll
    for (int t = 1; t < kAffTiles; ++t) {
        ulo[0] = fmin(ulo[0], lo[t][0]);
        ulo[1] = fmin(ulo[1], lo[t][1]);
        uhi[0] = fmax(uhi[0], hi[t][0]);
        uhi[1] = fmax(uhi[1], hi[t][1]);
    }
    double a1[kAffTiles], a2[kAffTiles], j11[kAffTiles], j12[kAffTiles];
#pragma unroll
    for (int t = 0; t < kAffTiles; ++t) a1[t] = a2[t] = j11[t] = j12[t] = 0.0;
    for (int64_t i = threadIdx.x; i < f.n_lens; i += 256) {
        const float4 l0 = f.lenses[i];
        const float4 l = moved_lens(l0, f.vel, i, f.time);
        const bool near_group = is_near(l0.x, l0.y, ulo, uhi, rn2);
#pragma unroll
        for (int t = 0; t < kAffTiles; ++t) {
            if (near_group && is_near(l0.x, l0.y, lo[t], hi[t], rn2)) continue;
            const double dx = c[t][0] - (double)l.x, dy = c[t][1] - (double)l.y, m = l.z;
            const double r2 = dx * dx + dy * dy;
            // 1 / r2: the hardware reciprocal refined by two Newton steps (to about 1 ulp), in
            // place of two IEEE divisions
            double inv = __builtin_amdgcn_rcp(r2);
            inv = fma(inv, fma(-r2, inv, 1.0), inv);
            inv = fma(inv, fma(-r2, inv, 1.0), inv);
            const double q = m * inv, q2 = q * inv;
            a1[t] += q * dx;
            a2[t] += q * dy;
            j11[t] += q2 * (dy * dy - dx * dx);
            j12[t] += -2.0 * q2 * dx * dy;
        }
    }
#pragma unroll
    for (int t = 0; t < kAffTiles; ++t) {
        if (t >= nt) break;
        red[0][threadIdx.x] = a1[t];
        red[1][threadIdx.x] = a2[t];
        red[2][threadIdx.x] = j11[t];
        red[3][threadIdx.x] = j12[t];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s)
                for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0 && f.affine) {
            double *o = f.affine + 8 * (size_t)tile[t];
            o[0] = red[0][0];
            o[1] = red[1][0];
            o[2] = red[2][0];
            o[3] = red[3][0];
            o[4] = -red[2][0];
        } else if (threadIdx.x == 0) {
            double *h = tile_hdr(f, tile[t]);
            h[0] = c[t][0];
            h[1] = c[t][1];
            h[2] = 0.5 * (hi[t][0] - lo[t][0]);
            h[3] = 0.5 * (hi[t][1] - lo[t][1]);
            h[4] = red[0][0];
            h[5] = red[1][0];
            h[6] = red[2][0];
            h[7] = red[3][0];
            h[8] = -red[2][0];
            h[9] = 1.0;
        }
        __syncthreads();   // red[] is reused by the next tile
    }
}

// ---------------------------------------------------------------- fit: exact far-field samples

// Workgroup (tile, part): 256 threads x 4 samples = samples [1024 part, 1024 (part + 1)).
// Samples come in groups g of 256: sample 64 (4 g + k) + i, k = 0..3, i = 0..63; thread i of wave w
// takes k = 0..3 of group 4 part + w.
// Direct sum over every lens with the near ones swapped for zero-mass padding, float32 runs
// of 16 lenses added four at a time in float32, then in FP64; writes the residual after the
// affine base (unnormalised).
// The four samples of a thread share one reciprocal per lens (simultaneous inversion of the
// product of their four squared distances: a far lens is at least r_near from every sample, so no
// product is zero).  Coordinates are staged scaled by 2^-4 (exact), which keeps that product in the
// float32 range for lenses up to about 1e6 from the samples (6.6e4 unscaled); a lens farther than
// that (its deflection there is below 1e-6 m) gets a zero reciprocal and is dropped.  The sums are
// scaled back by 2^4 with the FP64 combination.  The samples' error bound stays that of the plain path (far
// below the bfloat16 precision of the network they train).
// GRID: the samples of a thread share their first coordinate, so x - x_l and its square are
// computed once; every sample sees the same operations either way (the targets are
// bit-identical), and in every launch (the layout does not depend on the number of tiles).
__device__ __forceinline__ int sample_index(int part, int k, int tid)
{
    const int w = tid >> 6, lane = tid & 63;
    return (16 * part + 4 * w + k) * 64 + lane;
}

constexpr float kSampleScale = 0.0625f;   // 2^-4
// Zero-mass padding of the sample kernel, in its scaled coordinates: its squared distance (~2e18)
// keeps every pair product finite, so the quad product overflows to a zero reciprocal and every
// padding term is exactly 0 (never 0 x inf).
constexpr float kSamplePad = 1.0e9f;

template <bool GRID>
__global__ void __launch_bounds__(256) k_ff_samples(const FarArgs f, int parts)
{
    constexpr int LT = 256, T = 16, G = 4, S = 4;   // G runs of T lenses are added in float32, then in FP64
    static_assert(LT % (T * G) == 0, "tile shape");
    __shared__ float4 s_lens[2][LT];
    const uint32_t tile = blockIdx.x / (uint32_t)parts, part = blockIdx.x % (uint32_t)parts;
    double lo[2], hi[2], c[2], hw[2];
    int64_t i0[2];
    int n[2];
    tile_geom(f, tile, lo, hi, c, hw, i0, n);
    const double rn2 = f.r_near * f.r_near;
    const int tid = threadIdx.x;
    float px[S], py[S];   // sample positions (float32), scaled by 2^-4
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const int si = sample_index(part, k, tid);
        px[k] = (float)(c[0] + (double)f.samples[2 * si] * hw[0]) * kSampleScale;
        py[k] = (float)(c[1] + (double)f.samples[2 * si + 1] * hw[1]) * kSampleScale;
    }
    double A1[S] = {}, A2[S] = {};
    auto fetch = [&](int64_t i) -> float4 {
        if (i >= f.n_lens) return make_float4(kSamplePad, kSamplePad, 0.f, 0.f);
        const float4 l = f.lenses[i];
        return is_near(l.x, l.y, lo, hi, rn2) ? make_float4(kSamplePad, kSamplePad, 0.f, 0.f)
                                              : make_float4(l.x * kSampleScale, l.y * kSampleScale, l.z, l.w);
    };
    const int64_t n_tiles = (f.n_lens + LT - 1) / LT;
    float4 reg = n_tiles > 0 ? fetch(tid) : make_float4(0, 0, 0, 0);
    if (n_tiles > 0) s_lens[0][tid] = reg;
    __syncthreads();
    for (int64_t t = 0; t < n_tiles; ++t) {
        const int buf = (int)(t & 1);
        const bool more = t + 1 < n_tiles;
        if (more) reg = fetch((t + 1) * LT + tid);
        const float4 *L = s_lens[buf];
        for (int r = 0; r < LT; r += T * G) {
            float m1[S], m2[S];
#pragma unroll
            for (int h = 0; h < G; ++h) {
                float s1[S], s2[S];
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    const float4 l = L[r + h * T + j];
                    // GRID: the four samples share px[0]
                    const float dxs = px[0] - l.x, dxs2 = dxs * dxs;
                    float dx[S], dy[S], q[S];
#pragma unroll
                    for (int k = 0; k < S; ++k) {
                        dx[k] = GRID ? dxs : px[k] - l.x;
                        dy[k] = py[k] - l.y;
                        q[k] = fmaf(dy[k], dy[k], GRID ? dxs2 : dx[k] * dx[k]);
                    }
                    const float p01 = q[0] * q[1], p23 = q[2] * q[3];
                    const float g = l.z * __builtin_amdgcn_rcpf(p01 * p23);
                    const float g01 = g * p23, g23 = g * p01;
                    const float d[S] = {g01 * q[1], g01 * q[0], g23 * q[3], g23 * q[2]};
#pragma unroll
                    for (int k = 0; k < S; ++k) {
                        s1[k] = j == 0 ? d[k] * dx[k] : fmaf(d[k], dx[k], s1[k]);
                        s2[k] = j == 0 ? d[k] * dy[k] : fmaf(d[k], dy[k], s2[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    m1[k] = h == 0 ? s1[k] : m1[k] + s1[k];
                    m2[k] = h == 0 ? s2[k] : m2[k] + s2[k];
                }
            }
#pragma unroll
            for (int k = 0; k < S; ++k) {
                A1[k] += (double)m1[k];
                A2[k] += (double)m2[k];
            }
        }
        if (more) s_lens[buf ^ 1][tid] = reg;
        __syncthreads();
    }
    const double *h = tile_hdr(f, tile);
    const double a01 = h[4], a02 = h[5], j11 = h[6], j12 = h[7], j22 = h[8];
    // m (x - x_l) / r^2 of the scaled coordinates is 2^4 times the true term
    constexpr double kBack = kRcpBiasComp / 16.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const int si = sample_index(part, k, tid);
        const double d1 = (double)(px[k] * 16.0f) - c[0], d2 = (double)(py[k] * 16.0f) - c[1];
        const double r1 = A1[k] * kBack - (a01 + j11 * d1 + j12 * d2);
        const double r2 = A2[k] * kBack - (a02 + j12 * d1 + j22 * d2);
        float *out = f.targets + ((size_t)tile * f.n_samples + si) * 2;
        out[0] = (float)r1;
        out[1] = (float)r2;
        if (f.debug_targets) {
            float *dbg = f.debug_targets + ((size_t)tile * f.n_samples + si) * 2;
            dbg[0] = (float)r1;
            dbg[1] = (float)r2;
        }
    }
}

// Per tile: s_t = RMS of the residual samples (both components); targets /= s_t.
__global__ void __launch_bounds__(256) k_ff_normalize(const FarArgs f)
{
    __shared__ double red[256];
    const uint32_t tile = blockIdx.x;
    float *t = f.targets + (size_t)tile * f.n_samples * 2;
    double s = 0;
    for (int i = threadIdx.x; i < 2 * f.n_samples; i += 256) s += (double)t[i] * (double)t[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    double st = sqrt(red[0] / (2.0 * f.n_samples));
    if (!(st > 0.0)) st = 1.0;
    const float inv = (float)(1.0 / st);
    for (int i = threadIdx.x; i < 2 * f.n_samples; i += 256) t[i] *= inv;
    if (threadIdx.x == 0) tile_hdr(f, tile)[9] = st;
}

// ---------------------------------------------------------------- fit: training

// One workgroup of 8 waves (two per SIMD, so that one wave's MFMA, LDS and transcendental
// latencies hide behind the other's work) trains one tile's network with mini-batch Adam.  A step
// takes its batch in rounds of 256 samples, 32 per wave.  In a round every wave runs the forward
// and backward pass of its own samples (a lane pair per sample, as in the evaluation) and stages
// sample-major bfloat16 copies of h1, h2, dz2, dz1 and the features in LDS; after a workgroup
// barrier each wave contracts the blocks of the weight gradients it owns over all 256 samples
// (16x16x32 MFMAs whose operands come back through transposing LDS reads): the dW2 blocks of rows
// 16 (w / 2) .. + 16 and columns 32 (w % 2) .. + 32, and the dW1 rows 16 (w % 4) .. + 16 over the
// samples of waves 4 (w / 4) .. + 3.  The b2 and b1 gradients are the same contractions against a
// vector of ones (b2 split between the two waves of a row block, half of the samples each); the
// layer-3 gradients are summed by each wave over its own samples on the VALU, b3's per lane.  After
// the last round the partial sums are exchanged through LDS in a fixed order and each parameter is
// updated by the lane that owns its gradient: FP32 master weights and Adam moments live in the fit
// workspace (64.5 KB per tile, read and written once per step: the working set of the tiles in
// flight stays in L2; one 12-byte record per parameter), the bfloat16 weight copies the MFMAs read
// and the FP32 biases in LDS.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sample-major staging.  Row r (one sample) of a hidden-unit array holds the 64 units as eight
// 16-byte chunks of eight consecutive units, chunk c stored at position c ^ swz(r); a lane writes its
// 32 units (slots 8 g .. 8 g + 7 are the units 16 g + 8 hf + e, chunk 2 g + hf) as four chunks.  The
// swizzle puts the chunks of eight consecutive rows (one write instruction's first lanes) and the
// two chunks of four consecutive rows (one transposing read's group) on distinct banks.
__device__ __forceinline__ int swz(int r) { return ((r & 3) << 1) | ((r >> 2) & 1); }

__device__ __forceinline__ void stage_row(uint16_t *arr, int col, int hf, const uint32_t *w)
{
    uint8_t *row = reinterpret_cast<uint8_t *>(arr) + col * 128;
    const int sw = swz(col);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const u32x4 v = {w[4 * g], w[4 * g + 1], w[4 * g + 2], w[4 * g + 3]};
        *reinterpret_cast<u32x4 *>(row + (((2 * g + hf) ^ sw) << 4)) = v;
    }
}

using bf16x4 = __bf16 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;

// ds_read_b64_tr_b16: in each group of 16 lanes, element e of result lane 4 q + c is element c of the
// four bfloat16 values addressed by lane 4 e + q of the group.
__device__ __forceinline__ bf16x4 lds_tr4(const uint8_t *p)
{
    return __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4 *)(p));
}

// 16x16x32 MFMA operand of a staged hidden-unit array: unit 16 b + lane % 16, samples 8 (lane / 16)
// + 0 .. 7.  Lane 4 e + q of a group addresses units 16 b + 4 q .. + 3 of sample r = 8 (lane / 16)
// + 4 h + e, i.e. the 8-byte half q % 2 of chunk (2 b + q / 2) ^ swz(r).  With r % 4 = e and
// (r / 4) % 2 = h that is chunk 2 b ^ y0 ^ h of row r0 + 4 h, where the lane constants are
// r0 = 8 (lane / 16) + e and y0 = q / 2 ^ 2 e.
struct TrLane {
    int row0;   // byte offset of row r0 plus the lane's 8-byte half
    int y0;
};
__device__ __forceinline__ TrLane tr_lane(int lane)
{
    const int G = lane >> 4, s = lane & 15;
    return TrLane{(8 * G + (s >> 2)) * 128 + ((s & 1) << 3), ((s & 3) >> 1) ^ ((s >> 2) << 1)};
}
__device__ __forceinline__ bf16x8 tr_units(const uint16_t *arr, int b, const TrLane &t)
{
    const uint8_t *base = reinterpret_cast<const uint8_t *>(arr) + t.row0;
    const bf16x4 v0 = lds_tr4(base + (((2 * b) ^ t.y0) << 4));
    const bf16x4 v1 = lds_tr4(base + 512 + (((2 * b) ^ t.y0 ^ 1) << 4));
    return __builtin_shufflevector(v0, v1, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Feature rows: 16 values (32 bytes) per sample, chunk c (features 8 c .. 8 c + 7) of row r at
// position c ^ ((r >> 2) & 1).  Operand: feature lane % 16, samples 8 (lane / 16) + 0 .. 7.
__device__ __forceinline__ void stage_phi(uint16_t *arr, int col, int hf, const uint32_t *phi4)
{
    const u32x4 v = {phi4[0], phi4[1], phi4[2], phi4[3]};
    *reinterpret_cast<u32x4 *>(reinterpret_cast<uint8_t *>(arr) + col * 32 + ((hf ^ ((col >> 2) & 1)) << 4)) = v;
}
// (sample r = 8 (lane / 16) + 4 h + e, chunk q / 2 ^ h)
__device__ __forceinline__ bf16x8 tr_phi(const uint16_t *arr, int lane)
{
    const int G = lane >> 4, s = lane & 15, x = (s & 3) >> 1;
    const uint8_t *base = reinterpret_cast<const uint8_t *>(arr) + (8 * G + (s >> 2)) * 32 + ((s & 1) << 3);
    const bf16x4 v0 = lds_tr4(base + (x << 4));
    const bf16x4 v1 = lds_tr4(base + 128 + ((x ^ 1) << 4));
    return __builtin_shufflevector(v0, v1, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Optimiser state of one parameter: FP32 master weight and the two Adam moments, read and written
// as one 12-byte record.
struct AdamState {
    float w, m, v;
};

// Per-step factors of the optimiser, in FP64 and rounded once: the cosine-decayed learning rate
// lr (1 + cos(pi (t - 1) / S)) / 2 and the bias corrections 1 / (1 - beta^t) of step t (1-based).
__global__ void __launch_bounds__(256) k_adam_schedule(const FarArgs f)
{
    for (int t = (int)threadIdx.x + 1; t <= f.steps; t += 256) {
        f.sched[4 * (t - 1)] = (float)((double)f.lr * 0.5 * (1.0 + cos(3.14159265358979323846 * (t - 1) / f.steps)));
        f.sched[4 * (t - 1) + 3] = 0.f;
    }
    if (threadIdx.x == 0) {
        double b1t = 1.0, b2t = 1.0;
        for (int t = 1; t <= f.steps; ++t) {
            b1t *= 0.9;
            b2t *= 0.999;
            f.sched[4 * (t - 1) + 1] = (float)(1.0 / (1.0 - b1t));
            f.sched[4 * (t - 1) + 2] = (float)(1.0 / (1.0 - b2t));
        }
    }
}

constexpr int kTrainWaves = 8;
constexpr int kTrainThreads = 64 * kTrainWaves;
constexpr int kRoundSamples = 32 * kTrainWaves;
constexpr int kStageWords = 64 * 32;   // one [sample][unit] bfloat16 array of one wave

__global__ void __launch_bounds__(kTrainThreads) k_mlp_train(const FarArgs f)
{
    __shared__ __attribute__((aligned(16))) uint16_t Wbf[kNParamsPad];
    __shared__ __attribute__((aligned(16))) uint16_t W2T[64 * 64];
    __shared__ __attribute__((aligned(16))) float sbias[130];
    __shared__ __attribute__((aligned(16))) uint32_t sW3p[64];   // bfloat16 pair (W3[0][u], W3[1][u]) of unit u
    // array a (0 dz2, 1 h1, 2 dz1, 3 h2) of wave v at sstage + (a kTrainWaves + v) kStageWords
    __shared__ __attribute__((aligned(16))) uint16_t sstage[4 * kTrainWaves * kStageWords];
    __shared__ __attribute__((aligned(16))) uint16_t sphi[kTrainWaves][16 * 32];
    // per sample the bfloat16 terms of d3 = (o - t) / B: (hi0, hi1, lo0, lo1), d3 = hi + lo within 2^-18
    __shared__ __attribute__((aligned(16))) uint32_t sd3x[kTrainWaves][2 * 32];
    __shared__ __attribute__((aligned(16))) uint32_t szero[2];

    const uint32_t tile = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hf = lane >> 5, col = lane & 31;
    AdamState *ost = reinterpret_cast<AdamState *>(f.state) + (size_t)tile * kNParams;
    const float *tgt = f.targets + (size_t)tile * f.n_samples * 2;
    auto stg = [&](int a, int v) { return sstage + (a * kTrainWaves + v) * kStageWords; };

    for (int p = tid; p < kNParams; p += kTrainThreads) {
        const float w = f.init_params[p];
        ost[p] = AdamState{w, 0.f, 0.f};
        const uint16_t b = to_bf16(w);
        Wbf[wslot(p)] = b;
        if (p >= kOffW2 && p < kOffB2) W2T[m64((p - kOffW2) & 63, (p - kOffW2) >> 6)] = b;
        if (p >= kOffB1 && p < kOffW2) sbias[p - kOffB1] = w;
        if (p >= kOffB2 && p < kOffW3) sbias[64 + p - kOffB2] = w;
        if (p >= kOffW3 && p < kOffB3)
            reinterpret_cast<uint16_t *>(sW3p)[2 * ((p - kOffW3) & 63) + (p - kOffW3) / 64] = b;
        if (p >= kOffB3) sbias[128 + p - kOffB3] = w;
    }
    // (the first round's barrier orders these stores before their use)

    const int rounds = f.batch / kRoundSamples;
    const float inv_b = 1.0f / (float)f.batch;
    // owned blocks: dW2 rows 32 R .. + 32, columns 32 C .. + 32 (R, C from w % 4) and the dW1 rows
    // 16 (w % 4) .. + 16, both over the samples of waves 4 (w / 4) .. + 3; b2 of rows 32 R + 16 C .. + 16
    uint16_t *z2s = stg(0, wave), *h1s = stg(1, wave), *z1s = stg(2, wave), *h2s = stg(3, wave);
    uint32_t *d3x = sd3x[wave];
    if (tid < 2) szero[tid] = 0u;
    const u32x4 ones_u = {0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u};
    const bf16x8 ones = __builtin_bit_cast(bf16x8, ones_u);
    // the sample of the next round (samples of step t start at (t - 1) B mod N; B divides N), requested
    // a round ahead
    float u_n, t0_n, t1_n;
    auto fetch = [&](int base) __attribute__((always_inline)) {
        const int si = base + 32 * wave + col;
        u_n = f.samples[2 * si + hf];
        t0_n = tgt[2 * si];
        t1_n = tgt[2 * si + 1];
    };
    fetch(0);
    for (int step = 1, i0 = 0; step <= f.steps; ++step, i0 = (i0 + f.batch == f.n_samples) ? 0 : i0 + f.batch) {
        f32x4 g2[2][2] = {}, g1 = {}, gb1v = {}, gb2v = {};
        f32x4 w3m[4] = {}, gb3m = {};   // dW3 by unit block and b3: column lane % 16 < 4 holds d3 term n
        // owned weight-gradient blocks contracted over this round's samples, in wave order (the
        // operand addresses are recomputed here from laundered indices, not kept across the round)
        auto contract = [&]() __attribute__((always_inline)) {
            int cl = lane, cw = wave;
            asm volatile("" : "+v"(cl), "+v"(cw));
            const int r2 = (cw & 3) >> 1, c2 = cw & 1, tt = cw & 3, vv = 4 * (cw >> 2);
            const TrLane tl = tr_lane(cl);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                bf16x8 a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    a[i] = tr_units(stg(0, vv + v), 2 * r2 + i, tl);
                    b[i] = tr_units(stg(1, vv + v), 2 * c2 + i, tl);
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        g2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], g2[i][j], 0, 0, 0);
                gb2v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c2 ? a[1] : a[0], ones, gb2v, 0, 0, 0);
                const bf16x8 a1 = tr_units(stg(2, vv + v), tt, tl);
                const bf16x8 b1 = tr_phi(sphi[vv + v], cl);
                g1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, g1, 0, 0, 0);
                gb1v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, ones, gb1v, 0, 0, 0);
            }
        };
        for (int rd = 0;; ++rd) {
            // the staging area's readers of the previous round (or the last update's parameter
            // copies) are done
            __syncthreads();
            const float u = u_n, t0 = t0_n, t1 = t1_n;
            {
                const int nb = i0 + kRoundSamples * (rd + 1);
                fetch(nb == f.n_samples ? 0 : nb);
            }
            uint32_t phi4[4];
            features8(u, phi4);
            stage_phi(sphi[wave], col, hf, phi4);
            // forward: layer 1, layer 2 (each staged as soon as it is computed), layer 3
            float d1[32], d2[32];
            uint32_t h1[16], h2[16];
            const bf16x8 bphi = pack4(phi4);
            layer1<true>(Wbf, sbias, bphi, col, hf, d1, h1);
            stage_row(h1s, col, hf, h1);
            layer2<true>(Wbf, sbias, h1, col, hf, d2, h2);
            stage_row(h2s, col, hf, h2);
            float o0, o1;
            layer3_dot(Wbf, sbias, h2, hf, o0, o1);
            const float d30 = (o0 - t0) * inv_b, d31 = (o1 - t1) * inv_b;
            // dz2 = bf16(dh2 * silu'(z2)), dh2 = W3^T d3 as one 32x32x16 MFMA per output tile: d3 enters
            // as two bfloat16 terms hi + lo (equal to d3 within 2^-18 of it, far below the bfloat16
            // rounding of dz2), k = 0..3 = (hi0, hi1, lo0, lo1) against (W3[0][u], W3[1][u]) twice in
            // the rows of unit u (permuted like every hidden-producing layer, so the output registers
            // are the lane's slots); k >= 4 is zero
            const uint32_t d3hi = pk2(d30, d31);
            const uint32_t d3lo = pk2(d30 - lo_bf16(d3hi), d31 - hi_bf16(d3hi));
            const u32x4 bdv = {hf == 0 ? d3hi : 0u, hf == 0 ? d3lo : 0u, 0u, 0u};
            if (hf == 0) {
                using u32x2 = uint32_t __attribute__((ext_vector_type(2)));
                *reinterpret_cast<u32x2 *>(d3x + 2 * col) = u32x2{d3hi, d3lo};
            }
            uint32_t dz2[16];
#pragma unroll
            for (int T = 0; T < 2; ++T) {
                const uint32_t wp = hf == 0 ? sW3p[perm_row(32 * T + col)] : 0u;
                const u32x4 av = {wp, wp, 0u, 0u};
                const f32x16 acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                                           __builtin_bit_cast(bf16x8, bdv), f32x16{}, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 16; q += 2)
                    dz2[(16 * T + q) / 2] = pk2(acc[q] * d2[16 * T + q], acc[q + 1] * d2[16 * T + q + 1]);
            }
            stage_row(z2s, col, hf, dz2);
            // dh1 = W2^T dz2 (rows permuted like a hidden-producing layer), dz1 = bf16(dh1 * silu'(z1))
            uint32_t dz1[16];
#pragma unroll
            for (int T = 0; T < 2; ++T) {
                bf16x8 a[4];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) a[kk] = lds8(W2T + m64(perm_row(32 * T + col), 16 * kk + 8 * hf));
                sched_fence();
                f32x16 acc = {};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kk], pack4(dz2 + 4 * kk), acc, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 16; q += 2)
                    dz1[(16 * T + q) / 2] = pk2(acc[q] * d1[16 * T + q], acc[q + 1] * d1[16 * T + q + 1]);
            }
            stage_row(z1s, col, hf, dz1);
            // this wave's own staging: a wave-scope fence orders its stores and loads
            wave_sync();
            // dW3 and b3 over this wave's samples on the MFMA: A = h2 (unit 16 b + lane % 16, samples
            // 8 (lane / 16) ..), B = the samples' d3 terms in columns 0..3 and zeros elsewhere, read
            // transposed from the sample rows (lane 4 e + q of a group addresses the four terms of
            // sample 8 (lane / 16) + 4 h + e when q = 0, a zero block otherwise); b3 is the same B
            // against ones
            {
                int dl = lane, dw = wave;
                asm volatile("" : "+v"(dl), "+v"(dw));
                const uint16_t *h2s = stg(3, dw);
                const TrLane tl = tr_lane(dl);
                const int s16 = dl & 15;
                const uint8_t *row = reinterpret_cast<const uint8_t *>(sd3x[dw]) + (8 * (dl >> 4) + (s16 >> 2)) * 8;
                const uint8_t *zb = reinterpret_cast<const uint8_t *>(szero);
                const bool term = (s16 & 3) == 0;
                const bf16x4 v0 = lds_tr4(term ? row : zb), v1 = lds_tr4(term ? row + 32 : zb);
                const bf16x8 bd = __builtin_shufflevector(v0, v1, 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    w3m[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tr_units(h2s, b, tl), bd, w3m[b], 0, 0, 0);
                gb3m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ones, bd, gb3m, 0, 0, 0);
            }
            __syncthreads();   // every wave's staging of this round is complete
            if (rd + 1 == rounds) break;
            contract();
        }
        // From here to the end of the step the lane and wave indices are passed through an empty asm
        // statement, so that the addresses and indices derived from them are recomputed every step
        // (a few integer operations) instead of being kept, or spilled, across the rounds.
        int ln = lane, wv = wave;
        asm volatile("" : "+v"(ln), "+v"(wv));
        // The lane's parameters: slots 0-7 dW2 (tiles (i, w / 4) of its block), 8-11 dW1 (waves 0-3),
        // 12-15 the biases and layer-3 weights of unit 8 w + lane (lanes 0-7), slot 12 b3 (wave 0,
        // lanes 8 and 9); -1 = none.
        const int m16 = ln & 15, q4 = ln >> 4, own = wv >> 2;
        constexpr int kSlots = 16;
        int pid[kSlots];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            pid[k] = kOffW2 + 64 * (32 * ((wv & 3) >> 1) + 16 * (k >> 2) + 4 * q4 + (k & 3)) + 32 * (wv & 1) + 16 * own +
                     m16;
#pragma unroll
        for (int r = 0; r < 4; ++r) pid[8 + r] = wv < 4 ? kOffW1 + 16 * (16 * (wv & 3) + 4 * q4 + r) + m16 : -1;
        {
            const int un = 8 * wv + ln;
            pid[12] = ln < 8 ? kOffB1 + un : (wv == 0 && ln < 10 ? kOffB3 + ln - 8 : -1);
            pid[13] = ln < 8 ? kOffB2 + un : -1;
            pid[14] = ln < 8 ? kOffW3 + un : -1;
            pid[15] = ln < 8 ? kOffW3 + 64 + un : -1;
        }
        // the optimiser state of every slot is requested before the last round's contraction and the
        // exchange, so its global round trip overlaps them
        AdamState st[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) st[k] = ost[pid[k] < 0 ? 0u : (uint32_t)pid[k]];
        contract();
        // dW3 and b3 of output o = column o (hi term) + column o + 2 (lo term), held two lanes apart
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) w3m[b][r] += __shfl_down(w3m[b][r], 2);
        const float gb3 = gb3m[0] + __shfl_down(gb3m[0], 2);
        __syncthreads();   // the last round's readers are done: the staging area takes the partial sums
        float *xg1 = reinterpret_cast<float *>(sstage);    // [wave / 4][unit]: b1 partials
        float *xg2 = xg1 + 2 * 64;                         // [wave / 4][unit]: b2 partials
        float *xw3 = xg2 + 2 * 64;                         // [wave][o][unit]: dW3 partials
        float *x3 = xw3 + kTrainWaves * 2 * 64;            // [wave][o]: b3 partials
        float *x1 = x3 + kTrainWaves * 2;                  // [wave - 4][lane][4]: dW1 partials of waves 4-7
        float *x2 = x1 + 4 * 64 * 4;                       // [wave][lane][8]: dW2 tiles the wave does not own
        if ((ln & 15) == 0) {
            *reinterpret_cast<f32x4 *>(xg1 + own * 64 + 16 * (wv & 3) + 4 * (ln >> 4)) = gb1v;
            *reinterpret_cast<f32x4 *>(xg2 + own * 64 + 32 * ((wv & 3) >> 1) + 16 * (wv & 1) + 4 * (ln >> 4)) = gb2v;
        }
        if ((ln & 15) < 2) {
            // lane (G, o): units 16 b + 4 G + r
#pragma unroll
            for (int b = 0; b < 4; ++b)
                *reinterpret_cast<f32x4 *>(xw3 + (wv * 2 + (ln & 15)) * 64 + 16 * b + 4 * (ln >> 4)) = w3m[b];
        }
        if (ln < 2) x3[wv * 2 + ln] = gb3;
        if (wv >= 4) {
#pragma unroll
            for (int r = 0; r < 4; ++r) x1[((wv - 4) * 64 + ln) * 4 + r] = g1[r];
        }
        {
            // the partner wave (the other sample half of the same block) owns tiles (i, 1 - w / 4)
            f32x4 *o = reinterpret_cast<f32x4 *>(x2 + (wv * 64 + ln) * 8);
            o[0] = own ? g2[0][0] : g2[0][1];
            o[1] = own ? g2[1][0] : g2[1][1];
        }
        __syncthreads();
        float gr[kSlots];
        {
            const f32x4 *o = reinterpret_cast<const f32x4 *>(x2 + ((wv ^ 4) * 64 + ln) * 8);
            const f32x4 p0 = o[0], p1 = o[1];
            const f32x4 m0 = own ? g2[0][1] : g2[0][0], m1 = own ? g2[1][1] : g2[1][0];
            // half 0 (waves 0-3) first
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gr[r] = own ? p0[r] + m0[r] : m0[r] + p0[r];
                gr[4 + r] = own ? p1[r] + m1[r] : m1[r] + p1[r];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) gr[8 + r] = wv < 4 ? g1[r] + x1[(wv * 64 + ln) * 4 + r] : 0.f;
        if (ln < 8) {
            const int un = 8 * wv + ln;
            gr[12] = xg1[un] + xg1[64 + un];
            gr[13] = xg2[un] + xg2[64 + un];
            float s0 = 0.f, s1 = 0.f;
#pragma unroll
            for (int v = 0; v < kTrainWaves; ++v) {
                s0 += xw3[(v * 2 + 0) * 64 + un];
                s1 += xw3[(v * 2 + 1) * 64 + un];
            }
            gr[14] = s0;
            gr[15] = s1;
        } else {
            float g = 0.f;
            if (wv == 0 && ln < 10) {
#pragma unroll
                for (int v = 0; v < kTrainWaves; ++v) g += x3[v * 2 + ln - 8];
            }
            gr[12] = g;
            gr[13] = gr[14] = gr[15] = 0.f;
        }
        // Adam with bias correction and a cosine-decayed learning rate (the step's factors from the
        // schedule table); square root and quotient by the hardware instructions (1 ulp, far below
        // the bfloat16 rounding of the weights)
        const f32x4 sc = *reinterpret_cast<const f32x4 *>(f.sched + 4 * (step - 1));
        const float lr_t = sc[0], ibc1 = sc[1], ibc2 = sc[2];
        const bool dbg = f.debug_grad != nullptr && step == 1;
        float *dg = f.debug_grad + (size_t)tile * kNParams;
        auto adam = [&](const AdamState &s0, float g) __attribute__((always_inline)) {
            const float m = 0.9f * s0.m + 0.1f * g;
            const float v = 0.999f * s0.v + 0.001f * g * g;
            const float d = __builtin_amdgcn_sqrtf(v * ibc2) + 1e-8f;
            return AdamState{s0.w - lr_t * (m * ibc1) * __builtin_amdgcn_rcpf(d), m, v};
        };
        {
            // dW2 slots 4 i + r: row 32 R + 16 i + 4 q4 + r, column 32 C + 16 (w / 4) + m16; their LDS
            // positions in the swizzled W2 and W2T (see m64) follow from that structure
            const int q4b = q4 & 3, R = (wv & 3) >> 1;
            const int col2 = 32 * (wv & 1) + 16 * own + m16, rowb = 32 * R + 4 * q4b;
            const int cx = (col2 >> 3) ^ ((q4b & 2) << 1);
            const int y = (4 * R + (q4b >> 1)) ^ wsw(col2);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int i = k >> 2, r = k & 3;
                const int row = rowb + 16 * i + r;
                const int p = kOffW2 + 64 * row + col2;
                const AdamState s1 = adam(st[k], gr[k]);
                if (dbg) dg[p] = gr[k];
                ost[p] = s1;
                const uint16_t b = to_bf16(s1.w);
                Wbf[kOffW2 + 64 * row + (((cx ^ r) << 3) | (col2 & 7))] = b;
                W2T[col2 * 64 + (((y ^ (2 * i)) << 3) | (4 * (q4b & 1) + r))] = b;
            }
        }
        if (wv < 4) {
            // dW1 slots: rows 16 w + 4 q4 + r, feature m16
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = kOffW1 + 16 * (16 * (wv & 3) + 4 * q4 + r) + m16;
                const AdamState s1 = adam(st[8 + r], gr[8 + r]);
                if (dbg) dg[p] = gr[8 + r];
                ost[p] = s1;
                Wbf[p] = to_bf16(s1.w);
            }
        }
        if (ln < 8) {
            // b1, b2 and the two layer-3 weights of unit 8 w + lane
            const int un = 8 * wv + ln;
            const int ps[4] = {kOffB1 + un, kOffB2 + un, kOffW3 + un, kOffW3 + 64 + un};
            uint32_t w3pair = 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const AdamState s1 = adam(st[12 + k], gr[12 + k]);
                if (dbg) dg[ps[k]] = gr[12 + k];
                ost[ps[k]] = s1;
                const uint16_t b = to_bf16(s1.w);
                Wbf[ps[k]] = b;
                if (k < 2) sbias[64 * k + un] = s1.w;
                else w3pair |= (uint32_t)b << (16 * (k - 2));
            }
            sW3p[un] = w3pair;
        } else if (wv == 0 && ln < 10) {
            const int p = kOffB3 + ln - 8;
            const AdamState s1 = adam(st[12], gr[12]);
            if (dbg) dg[p] = gr[12];
            ost[p] = s1;
            Wbf[p] = to_bf16(s1.w);
            sbias[128 + ln - 8] = s1.w;
        }
    }
    __syncthreads();
    // the fitted network: bfloat16 weights and FP32 biases (biases kept at full precision)
    uint16_t *wout = tile_w(f, tile);
    float *bout = reinterpret_cast<float *>(reinterpret_cast<uint8_t *>(wout) + kTileBiasOff);
    for (int p = tid; p < kNParams; p += kTrainThreads) wout[p] = Wbf[wslot(p)];
    for (int p = tid; p < 130; p += kTrainThreads) bout[p] = sbias[p];
}

// ---------------------------------------------------------------- eval: cell grid

__device__ __forceinline__ int cell_of(const CellArgs &g, float x, float y)
{
    const double fx = floor(((double)x - g.ox) / g.cs), fy = floor(((double)y - g.oy) / g.cs);
    if (!(fx >= 0.0 && fx < (double)g.ncx && fy >= 0.0 && fy < (double)g.ncy)) return -1;
    return (int)fy * g.ncx + (int)fx;
}

__global__ void k_cells_count(const CellArgs g)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n_lens; i += stride) {
        const float4 l = g.lenses[i];
        const int c = cell_of(g, l.x, l.y);
        if (c >= 0) atomicAdd(&g.count[c], 1);
    }
}

// Exclusive scan of count[0 .. n_cells) into start[0 .. n_cells] with one workgroup.
__global__ void __launch_bounds__(1024) k_cells_scan(const CellArgs g)
{
    __shared__ int part[1024];
    const int n = g.n_cells, tid = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int b = min(n, tid * per), e = min(n, b + per);
    int s = 0;
    for (int i = b; i < e; ++i) s += g.count[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int i = b; i < e; ++i) {
        g.start[i] = run;
        run += g.count[i];
    }
    if (tid == 1023) g.start[n] = part[1023];
}

__global__ void k_cells_fill(const CellArgs g)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n_lens; i += stride) {
        const float4 l = g.lenses[i];
        const int c = cell_of(g, l.x, l.y);
        if (c >= 0) g.idx[g.start[c] + atomicAdd(&g.cursor[c], 1)] = (int)i;
    }
}

// Lens indices of every cell in increasing order, so the near-field order is deterministic.
__global__ void k_cells_sort(const CellArgs g)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.n_cells) return;
    const int b = g.start[c], e = g.start[c + 1];
    for (int i = b + 1; i < e; ++i) {
        const int v = g.idx[i];
        int j = i - 1;
        while (j >= b && g.idx[j] > v) {
            g.idx[j + 1] = g.idx[j];
            --j;
        }
        g.idx[j + 1] = v;
    }
}

// ---------------------------------------------------------------- eval: surrogate

// `splits` workgroups per fit tile, workgroup q taking passes q, q + splits, ... of the tile's
// rays (every ray is computed the same way whatever the split).  Rays go 128 at a time (32 per
// wave, a lane pair per ray): far
// field from the affine base plus the network (layers 1-2 on MFMA), near field summed exactly
// over the candidate lenses of the cells around the tile (far ones masked to zero-mass
// padding), the two lanes of a ray splitting the lenses; then the FP64 lens equation and
// wave-aggregated binning into the job's map.
template <bool DUMP>
__global__ void __launch_bounds__(256) k_surrogate(const FarArgs f, const CellArgs g, int splits)
{
    constexpr int CAP = 2048, T = 16;
    __shared__ __attribute__((aligned(16))) uint16_t Wbf[kNParamsPad];
    __shared__ __attribute__((aligned(16))) float sbias[130];
    __shared__ float4 s_near[CAP];
    __shared__ __attribute__((aligned(16))) uint32_t s_zero[4];
    __shared__ int s_cells[4];
    __shared__ uint32_t s_lost;

    const uint32_t item = blockIdx.x / (uint32_t)splits, split = blockIdx.x % (uint32_t)splits;
    const uint32_t tile = f.eval_tiles ? (uint32_t)f.eval_tiles[item] : item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hf = lane >> 5, col = lane & 31;
    double lo[2], hi[2], c[2], hw[2];
    int64_t i0[2];
    int n[2];
    tile_geom(f, tile, lo, hi, c, hw, i0, n);
    const double *hd = tile_hdr(f, tile);
    // a moving field uses the affine base refreshed at f.time; the network residual is the fitted one
    const double *ab = f.affine ? f.affine + 8 * (size_t)tile : hd + 4;
    const double a01 = ab[0], a02 = ab[1], j11 = ab[2], j12 = ab[3], j22 = ab[4], st = hd[9];
    const uint16_t *wsrc = tile_w(f, tile);
    const float *bsrc = reinterpret_cast<const float *>(reinterpret_cast<const uint8_t *>(wsrc) + kTileBiasOff);
    for (int p = tid; p < kNParams; p += 256) Wbf[wslot(p)] = wsrc[p];
    for (int p = tid; p < 130; p += 256) sbias[p] = bsrc[p];
    if (tid < 4) s_zero[tid] = 0u;
    if (tid == 0) {
        s_lost = 0u;
        // candidate cells: those overlapping the tile rectangle grown by r_near
        s_cells[0] = max(0, (int)floor((lo[0] - f.r_near - g.ox) / g.cs));
        s_cells[1] = min(g.ncx - 1, (int)floor((hi[0] + f.r_near - g.ox) / g.cs));
        s_cells[2] = max(0, (int)floor((lo[1] - f.r_near - g.oy) / g.cs));
        s_cells[3] = min(g.ncy - 1, (int)floor((hi[1] + f.r_near - g.oy) / g.cs));
    }
    __syncthreads();
    const int cx0 = s_cells[0], cx1 = s_cells[1], cy0 = s_cells[2], cy1 = s_cells[3];
    const int ncx = max(0, cx1 - cx0 + 1);
    const int n_rows = max(0, cy1 - cy0 + 1);
    // candidate lenses are the concatenation of cell rows cy0..cy1, each the contiguous index
    // range start[cy * ncx_grid + cx0] .. start[cy * ncx_grid + cx1 + 1]
    int n_cand = 0;
    for (int r = 0; r < n_rows; ++r) {
        const int row = (cy0 + r) * g.ncx;
        n_cand += g.start[row + cx1 + 1] - g.start[row + cx0];
    }
    const double rn2 = f.r_near * f.r_near;
    const int n_batches = (n_cand + CAP - 1) / CAP;

    // stage candidates [b CAP, b CAP + CAP) (far ones become zero-mass padding)
    auto stage = [&](int b) {
        const int base = b * CAP;
        for (int k = tid; k < CAP; k += 256) {
            float4 v = make_float4(kPadCoord, kPadCoord, 0.f, 0.f);
            int e = base + k;
            if (e < n_cand) {
                for (int r = 0; r < n_rows; ++r) {
                    const int row = (cy0 + r) * g.ncx;
                    const int len = g.start[row + cx1 + 1] - g.start[row + cx0];
                    if (e < len) {
                        // near set by fit-time position; a moving lens enters at its position at f.time
                        const int li = g.idx[g.start[row + cx0] + e];
                        const float4 l = g.lenses[li];
                        if (is_near(l.x, l.y, lo, hi, rn2)) v = moved_lens(l, f.vel, li, f.time);
                        break;
                    }
                    e -= len;
                }
            }
            s_near[k] = v;
        }
    };
    if (n_batches == 1) stage(0);
    __syncthreads();

    const int n_rays = n[0] * n[1];
    const int passes = (f.TX * f.TY + 127) / 128;
    for (int ps = (int)split; ps < passes; ps += splits) {
        const int ri = 128 * ps + 32 * wave + col;
        const int ix = ri % f.TX, iy = ri / f.TX;
        const bool active = ri < f.TX * f.TY && ix < n[0] && iy < n[1];
        const int64_t g1 = i0[0] + ix, g2 = i0[1] + iy, rg = g2 * f.gn1 + g1;
        const float x1 = ray_coord(f.glo1, f.gt1, g1, f.jitter ? jitter_u(f.jkey1, rg) : 0.5);
        const float x2 = ray_coord(f.glo2, f.gt2, g2, f.jitter ? jitter_u(f.jkey2, rg) : 0.5);
        // far field: network
        float o0 = 0.f, o1 = 0.f;
        if (!f.affine_only) {
            const float u = hf == 0 ? (float)(((double)x1 - c[0]) / hw[0]) : (float)(((double)x2 - c[1]) / hw[1]);
            uint32_t phi4[4];
            features8(u, phi4);
            Fwd fw;
            forward32<false>(Wbf, sbias, reinterpret_cast<const uint16_t *>(s_zero), phi4, lane, fw);
            o0 = fw.o[0];
            o1 = fw.o[1];
        }
        // near field: this lane takes half hf of every staged batch
        double A1 = 0.0, A2 = 0.0;
        for (int b = 0; b < n_batches; ++b) {
            if (n_batches > 1) {
                __syncthreads();
                stage(b);
                __syncthreads();
            }
            // the two lanes of a ray split the batch: [0, half) and [half, nb), in runs of T
            const int nb = min(CAP, n_cand - b * CAP);
            const int half = ((nb + 1) / 2 + T - 1) / T * T;
            const float4 *L = s_near + (hf ? half : 0);
            const int m = hf ? max(0, nb - half) : min(half, nb);
            const int mr = (m + T - 1) / T * T;
            for (int r = 0; r < mr; r += T) {
                float s1 = 0.f, s2 = 0.f;
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    const float4 l = L[r + j];
                    const float dx = x1 - l.x, dy = x2 - l.y;
                    const float d = l.z * __builtin_amdgcn_rcpf(fmaf(dy, dy, dx * dx));
                    s1 = fmaf(d, dx, s1);
                    s2 = fmaf(d, dy, s2);
                }
                A1 += (double)s1;
                A2 += (double)s2;
            }
        }
        const double B1 = __shfl_xor(A1, 32), B2 = __shfl_xor(A2, 32);
        const double N1 = (hf == 0 ? A1 + B1 : B1 + A1) * kRcpBiasComp;
        const double N2 = (hf == 0 ? A2 + B2 : B2 + A2) * kRcpBiasComp;
        const double d1 = (double)x1 - c[0], d2 = (double)x2 - c[1];
        const double F1 = a01 + j11 * d1 + j12 * d2 + st * (double)o0;
        const double F2 = a02 + j12 * d1 + j22 * d2 + st * (double)o1;
        const double y1 = f.lam1 * (double)x1 - (F1 + N1);
        const double y2 = f.lam2 * (double)x2 - (F2 + N2);
        int key = -2;
        if (active && hf == 0) {
            const double p1 = floor((y1 - f.mlo1) * f.ms1), p2 = floor((y2 - f.mlo2) * f.ms2);
            key = (p1 >= 0.0 && p1 < (double)f.mn1 && p2 >= 0.0 && p2 < (double)f.mn2) ? (int)p2 * f.mn1 + (int)p1 : -1;
            if (DUMP) {
                const int64_t rw = (i0[1] + iy - f.wlo2) * f.wn1 + (i0[0] + ix - f.wlo1);
                f.ray_y[2 * rw] = y1;
                f.ray_y[2 * rw + 1] = y2;
                f.ray_pix[rw] = key;
            }
        }
        // runs of equal keys over consecutive lanes are added once
        const int prev = __shfl_up(key, 1);
        const bool head = (lane == 0) || (key != prev);
        const unsigned long long H = __ballot(head);
        const unsigned long long above = lane == 63 ? 0ull : (H >> (lane + 1));
        const int nxt = above ? lane + 1 + __builtin_ctzll(above) : 64;
        if (head && key >= 0) atomicAdd(&f.counts[key], (uint32_t)(nxt - lane));
        if (head && key == -1) atomicAdd(&s_lost, (uint32_t)(nxt - lane));
    }
    (void)n_rays;
    __syncthreads();
    if (tid == 0 && s_lost) atomicAdd(f.lost, (unsigned long long)s_lost);
}

__global__ void k_write_model_header(uint8_t *model, uint64_t hash, int64_t n_tiles, int tiles_x, int tiles_y, int TX,
                                     int TY)
{
    uint64_t *h = reinterpret_cast<uint64_t *>(model);
    h[0] = kModelMagic;
    h[1] = hash;
    h[2] = (uint64_t)n_tiles;
    int32_t *d = reinterpret_cast<int32_t *>(model + 24);
    d[0] = tiles_x;
    d[1] = tiles_y;
    d[2] = TX;
    d[3] = TY;
    h[5] = 0;   // lens checksum, added by k_lens_checksum
}

// *out += sum over lens records i of mix64(bits of (x1, x2) + (i + 1) G) + mix64(bits of (m, pad) ^ i):
// a checksum of the lens array that does not depend on the order of the additions (wrapping
// 64-bit sums), one atomic per wave.
__global__ void __launch_bounds__(256) k_lens_checksum(const float4 *lenses, int64_t n, unsigned long long *out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint4 v = reinterpret_cast<const uint4 *>(lenses)[i];
        const uint64_t a = ((uint64_t)v.y << 32) | v.x, b = ((uint64_t)v.w << 32) | v.z;
        acc += mix64(a + (uint64_t)(i + 1) * kGolden) + mix64(b ^ (uint64_t)i);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

}  // namespace

hipError_t launch_lens_checksum(const float4 *lenses, int64_t n, unsigned long long *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(2048, (n + 255) / 256);
    hipLaunchKernelGGL(k_lens_checksum, dim3((unsigned)blocks), dim3(256), 0, s, lenses, n, out);
    return hipGetLastError();
}

// affine bases of `count` tiles: four per workgroup once there are at least 8192 (2048
// workgroups), else one per workgroup (the sums are the same either way)
hipError_t launch_affine(const FarArgs &f, int64_t count, hipStream_t s)
{
    if (count >= 8192)
        hipLaunchKernelGGL(k_ff_affine<4>, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, s, f);
    else
        hipLaunchKernelGGL(k_ff_affine<1>, dim3((unsigned)count), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_ff_fit(const FarArgs &f, uint64_t hash, hipStream_t s)
{
    const uint32_t nt = (uint32_t)f.n_tiles;
    hipLaunchKernelGGL(k_write_model_header, dim3(1), dim3(1), 0, s, f.model, hash, f.n_tiles, f.tiles_x, f.tiles_y,
                       f.TX, f.TY);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_lens_checksum(f.lenses, f.n_lens, reinterpret_cast<unsigned long long *>(f.model + 40), s)) !=
        hipSuccess)
        return e;
    if ((e = launch_affine(f, nt, s)) != hipSuccess) return e;
    const int parts = f.n_samples / 1024;
    if (f.grid_samples)
        hipLaunchKernelGGL(k_ff_samples<true>, dim3(nt * (uint32_t)parts), dim3(256), 0, s, f, parts);
    else
        hipLaunchKernelGGL(k_ff_samples<false>, dim3(nt * (uint32_t)parts), dim3(256), 0, s, f, parts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ff_normalize, dim3(nt), dim3(256), 0, s, f);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (f.steps > 0) {
        hipLaunchKernelGGL(k_adam_schedule, dim3(1), dim3(256), 0, s, f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_mlp_train, dim3(nt), dim3(kTrainThreads), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_ff_eval(const FarArgs &f, const CellArgs &g, hipStream_t s)
{
    hipError_t e;
    const int cb = (int)std::min<int64_t>(4096, (g.n_lens + 255) / 256 + 1);
    hipLaunchKernelGGL(k_cells_count, dim3(cb), dim3(256), 0, s, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cells_scan, dim3(1), dim3(1024), 0, s, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cells_fill, dim3(cb), dim3(256), 0, s, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cells_sort, dim3((g.n_cells + 255) / 256), dim3(256), 0, s, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const uint32_t grid = (uint32_t)(f.eval_tiles ? f.n_eval : f.n_tiles);
    if (grid == 0) return hipSuccess;
    if (f.affine) {
        if ((e = launch_affine(f, grid, s)) != hipSuccess) return e;
    }
    // large tiles are few: split their rays over up to 8 workgroups so that about 4096 run
    const int passes = (f.TX * f.TY + 127) / 128;
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>({8, passes, (4096 + grid - 1) / grid}));
    if (f.ray_y)
        hipLaunchKernelGGL((k_surrogate<true>), dim3(grid * (uint32_t)splits), dim3(256), 0, s, f, g, splits);
    else
        hipLaunchKernelGGL((k_surrogate<false>), dim3(grid * (uint32_t)splits), dim3(256), 0, s, f, g, splits);
    return hipGetLastError();
}

}  // namespace rs
