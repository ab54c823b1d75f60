// tri_fft.hip -- the pressure step around the Poisson wavenumber solves
// (Sec. 2.2): spanwise real FFT of the divergence of the intermediate
// velocity, inverse FFT of the pseudo-pressure, gradient correction; for the
// 3-D step also the streamwise cosine transform (at the end of the file).
//
// Layout: fields [Nz][Ny][Nx] FP64, x fastest.  A spanwise line is one
// (j, i) station; the Ny*Nx stations of a z-plane are contiguous, so the
// `lines` stations g = j*Nx + i of every plane form one row of `lines`
// doubles.  Spectra are [Nz/2+1][Ny][Nx] complex (interleaved re, im).
//
// Real FFT of N = 2M points through one complex FFT of M points:
// z_n = x_{2n} + i x_{2n+1}, Z = DFT_M(z), E_k = (Z_k + conj Z_{M-k})/2,
// O_k = (Z_k - conj Z_{M-k})/(2i), X_k = E_k + W^k O_k and
// X_{M-k} = conj(E_k - W^k O_k), W = exp(-2 pi i/N).  The inverse runs the
// same algebra backwards (E_k = (X_k + conj X_{M-k})/2,
// O_k = (X_k - conj X_{M-k}) W^{-k}/2, Z_k = E_k + i O_k) and an inverse
// complex FFT as conj(DFT_M(conj Z))/M; the imaginary parts of X_0 and X_M
// are ignored (they are zero for the spectrum of a real line).
//
// The complex FFT is a self-sorting mixed-radix (4, 2, 3, 5; 8 as well for
// the cosine transform) Stockham
// transform held in LDS: a workgroup takes L neighbouring lines (L doubles
// per plane row, coalesced), T = 256/L threads per line; in every pass a
// thread reads its butterflies' inputs into registers, the workgroup
// synchronises, and the thread writes the outputs to their sorted places
// (one buffer, two barriers per pass).  The transform is bound by HBM: each
// element is read once and written once.
#include <algorithm>
#include <cstdlib>

#include "tri_internal.h"
#include "tri_ns.h"

namespace tri {
namespace {

struct cplx {
    double re, im;
};
typedef double v2d __attribute__((ext_vector_type(2)));

__device__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cconj(cplx a) { return {a.re, -a.im}; }
__device__ inline cplx cmul_mi(cplx a) { return {a.im, -a.re}; }   // -i * a

// Forward DFTs of length R in place (exp(-2 pi i k m / R)).
template <int R>
__device__ inline void dft(cplx *v);

template <>
__device__ inline void dft<2>(cplx *v)
{
    const cplx a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <>
__device__ inline void dft<3>(cplx *v)
{
    constexpr double s3 = 0.86602540378443864676;   // sin(2 pi/3)
    const cplx s = cadd(v[1], v[2]);
    const cplx d = csub(v[1], v[2]);
    const cplx t = {v[0].re - 0.5 * s.re, v[0].im - 0.5 * s.im};
    const cplx u = {s3 * d.im, -s3 * d.re};              // -i sin(2 pi/3) (x1 - x2)
    v[0] = cadd(v[0], s);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
}

template <>
__device__ inline void dft<4>(cplx *v)
{
    const cplx a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const cplx c = cadd(v[1], v[3]), d = cmul_mi(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
}

template <>
__device__ inline void dft<5>(cplx *v)
{
    constexpr double c1 = 0.30901699437494742410;    // cos(2 pi/5)
    constexpr double c2 = -0.80901699437494742410;   // cos(4 pi/5)
    constexpr double s1 = 0.95105651629515357212;    // sin(2 pi/5)
    constexpr double s2 = 0.58778525229247312917;    // sin(4 pi/5)
    const cplx a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const cplx a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const cplx x0 = v[0];
    const cplx p1 = {x0.re + c1 * a1.re + c2 * a2.re, x0.im + c1 * a1.im + c2 * a2.im};
    const cplx p2 = {x0.re + c2 * a1.re + c1 * a2.re, x0.im + c2 * a1.im + c1 * a2.im};
    const cplx q1 = cmul_mi({s1 * b1.re + s2 * b2.re, s1 * b1.im + s2 * b2.im});
    const cplx q2 = cmul_mi({s2 * b1.re - s1 * b2.re, s2 * b1.im - s1 * b2.im});
    v[0] = cadd(x0, cadd(a1, a2));
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
}

template <>
__device__ inline void dft<8>(cplx *v)
{
    // two radix-4 transforms of the even and odd elements, joined by W_8^k
    constexpr double h = 0.70710678118654752440;   // 1/sqrt(2)
    cplx e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e);
    dft<4>(o);
    const cplx o1 = {h * (o[1].re + o[1].im), h * (o[1].im - o[1].re)};     // W_8 o1
    const cplx o2 = cmul_mi(o[2]);                                          // W_8^2 o2
    const cplx o3 = {h * (o[3].im - o[3].re), -h * (o[3].im + o[3].re)};    // W_8^3 o3
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

// Radix 16 = 4 x 4 and radix 9 = 3 x 3 in registers: X[k1 + R1 k2] =
// DFT_R2 over b of W_R^{b k1} DFT_R1(v_b, v_{b+R2}, ...)[k1].
template <>
__device__ inline void dft<16>(cplx *v)
{
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;   // cos, sin(pi/8)
    constexpr double h = 0.70710678118654752440;
    const cplx tw[3][3] = {{{c1, -s1}, {h, -h}, {s1, -c1}},      // W_16^{b k1}, b = 1..3, k1 = 1..3
                           {{h, -h}, {0.0, -1.0}, {-h, -h}},
                           {{s1, -c1}, {-h, -h}, {-c1, s1}}};
    cplx y[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int a = 0; a < 4; ++a) y[b][a] = v[b + 4 * a];
        dft<4>(y[b]);
    }
#pragma unroll
    for (int b = 1; b < 4; ++b)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) y[b][k1] = cmul(y[b][k1], tw[b - 1][k1 - 1]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        dft<4>(z);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = z[k2];
    }
}

template <>
__device__ inline void dft<9>(cplx *v)
{
    constexpr double c1 = 0.76604444311897803520, s1 = 0.64278760968653932632;   // cos, sin(2 pi/9)
    constexpr double c2 = 0.17364817766693034885, s2 = 0.98480775301220805936;   // 4 pi/9
    constexpr double c4 = -0.93969262078590838405, s4 = 0.34202014332566873304;  // 8 pi/9
    const cplx tw[2][2] = {{{c1, -s1}, {c2, -s2}}, {{c2, -s2}, {c4, -s4}}};      // W_9^{b k1}
    cplx y[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
#pragma unroll
        for (int a = 0; a < 3; ++a) y[b][a] = v[b + 3 * a];
        dft<3>(y[b]);
    }
#pragma unroll
    for (int b = 1; b < 3; ++b)
#pragma unroll
        for (int k1 = 1; k1 < 3; ++k1) y[b][k1] = cmul(y[b][k1], tw[b - 1][k1 - 1]);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        cplx z[3] = {y[0][k1], y[1][k1], y[2][k1]};
        dft<3>(z);
#pragma unroll
        for (int k2 = 0; k2 < 3; ++k2) v[k1 + 3 * k2] = z[k2];
    }
}

constexpr int kFftThreads = 256;

// Twiddle W_M^q from a full table (M entries) or from two short ones
// (W^q = W^{64 (q >> 6)} W^{q & 63}: 64 + M/64 entries, for long transforms).
// With TwSplit a butterfly looks up W^a once and forms W^{ra} as powers.
struct TwFull {
    static constexpr bool kPowers = false;
    const cplx *t;
    __device__ cplx operator()(int q) const { return t[q]; }
};
struct TwSplit {
    static constexpr bool kPowers = true;
    const cplx *lo, *hi;
    __device__ cplx operator()(int q) const { return cmul(hi[q >> 6], lo[q & 63]); }
};

// Element i of a line sits at slot i of buf[][L], or, with PAD, at slot
// i + i/16: with few lines a workgroup (the streamwise rows) the first passes
// write with lane strides of R elements, which without the padding fall on the
// same LDS banks.
template <bool PAD>
__device__ __forceinline__ int fft_slot(int i)
{
    return PAD ? i + (i >> 4) : i;
}

// One Stockham pass of radix R over the M-point transforms of the L lines in
// buf[M][L].  Butterfly j reads elements j + r M/R, twiddles element r by
// W_{Ns R}^{(j mod Ns) r} = twM((j mod Ns) r M/(Ns R)), and writes output r to
// (j/Ns) Ns R + (j mod Ns) + r Ns.
template <int R, int IT, class TW, bool PAD = false>
__device__ inline void fft_pass(cplx *buf, const TW &twM, int M, int Ns, int L, int ln, int tr, int T)
{
    const int nb = M / R;
    const int tws = M / (Ns * R);
    cplx v[IT][R];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int j = tr + it * T;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = buf[fft_slot<PAD>(j + r * nb) * L + ln];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int j = tr + it * T;
        if (j < nb) {
            const int jn = j % Ns;
            if (TW::kPowers) {
                const cplx w1 = twM(jn * tws);
                cplx wr = w1;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    v[it][r] = cmul(v[it][r], wr);
                    wr = cmul(wr, w1);
                }
            } else {
#pragma unroll
                for (int r = 1; r < R; ++r) v[it][r] = cmul(v[it][r], twM(jn * r * tws));
            }
            dft<R>(v[it]);
            const int d = (j / Ns) * Ns * R + jn;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[fft_slot<PAD>(d + r * Ns) * L + ln] = v[it][r];
        }
    }
    __syncthreads();
}

constexpr int kRadix8 = 1, kRadix16 = 2;

// RSET: which long radices are compiled in (kRadix8, kRadix16 for 16 and 9),
// only where the plan uses them: their registers would otherwise lower the
// occupancy of every transform kernel.
template <int L, int MMAX, int RSET, class TW, bool PAD = false>
__device__ inline void fft_lines(cplx *buf, const TW &twM, const FftShape &S, int ln, int tr)
{
    constexpr int T = kFftThreads / L;
    int Ns = 1;
    for (int s = 0; s < S.npass; ++s) {
        switch (S.radix[s]) {
        case 16:
            if constexpr ((RSET & kRadix16) != 0)
                fft_pass<16, (MMAX / 16 + T - 1) / T, TW, PAD>(buf, twM, S.M, Ns, L, ln, tr, T);
            break;
        case 9:
            if constexpr ((RSET & kRadix16) != 0)
                fft_pass<9, (MMAX / 9 + T - 1) / T, TW, PAD>(buf, twM, S.M, Ns, L, ln, tr, T);
            break;
        case 8:
            if constexpr ((RSET & kRadix8) != 0)
                fft_pass<8, (MMAX / 8 + T - 1) / T, TW, PAD>(buf, twM, S.M, Ns, L, ln, tr, T);
            break;
        case 4: fft_pass<4, (MMAX / 4 + T - 1) / T, TW, PAD>(buf, twM, S.M, Ns, L, ln, tr, T); break;
        case 2: fft_pass<2, (MMAX / 2 + T - 1) / T, TW, PAD>(buf, twM, S.M, Ns, L, ln, tr, T); break;
        case 3: fft_pass<3, (MMAX / 3 + T - 1) / T, TW, PAD>(buf, twM, S.M, Ns, L, ln, tr, T); break;
        default: fft_pass<5, (MMAX / 5 + T - 1) / T, TW, PAD>(buf, twM, S.M, Ns, L, ln, tr, T); break;
        }
        Ns *= S.radix[s];
    }
}

// twM[q] = W_M^q (q < M), twN[k] = W_N^{k} (k <= M/2), W_n = exp(-2 pi i/n).
__device__ inline void make_twiddles(cplx *twM, cplx *twN, int M)
{
    for (int q = threadIdx.x; q < M; q += kFftThreads) {
        double s, c;
        sincospi(2.0 * q / M, &s, &c);
        twM[q] = {c, -s};
    }
    for (int k = threadIdx.x; k <= M / 2; k += kFftThreads) {
        double s, c;
        sincospi((double)k / M, &s, &c);
        twN[k] = {c, -s};
    }
}

// Rows a thread loads (at most) and rows per batch of loads issued together:
// the loads of a batch are all in flight before the first is used.
template <int L, int MMAX>
struct FftTile {
    static constexpr int T = kFftThreads / L;
    static constexpr int NPT = (2 * MMAX + T - 1) / T;          // rows k = tr + u T < Nz
    static constexpr int KP = (MMAX / 2 + 1 + T - 1) / T;        // mode pairs k = tr + u T <= M/2
    static constexpr int NB = 12;
};

// Forward: x rows (DIV = 0), or the divergence of (v, w) (DIV = 1) or of
// (u, v, w) (DIV = 2) -> spectrum rows.
template <int L, int MMAX, int DIV, int RSET>
__global__ void __launch_bounds__(kFftThreads) k_rfft_z(FftArgs A)
{
    using TL = FftTile<L, MMAX>;
    constexpr int T = TL::T, NPT = TL::NPT, NB = DIV == 2 ? 8 : TL::NB;
    extern __shared__ double lds_fft[];
    const int M = A.S.M;
    cplx *buf = reinterpret_cast<cplx *>(lds_fft);   // [M][L]
    cplx *twM = buf + (size_t)M * L;                 // [M]
    cplx *twN = twM + M;                             // [M/2 + 1]
    const int ln = threadIdx.x % L, tr = threadIdx.x / L;
    int64_t blk = blockIdx.x;
    if (DIV == 2) {
        // The x-face rows of u hold Nx+1 values, so a chunk of L stations
        // reads L+1 faces spanning two cache lines, the second shared with the
        // next chunk of the row.  Workgroups are dealt to the 8 XCDs in turn:
        // each XCD takes a contiguous run of chunks of every row, walking the
        // rows in order, so that both readers of such a line, and of the v
        // faces shared with the next row, are resident in one L2 together.
        const int cpr = A.Nx / L;
        if (A.Nx % L == 0 && cpr % 8 == 0) {
            const int64_t wr = cpr / 8, x = blk % 8, s = blk / 8;
            blk = (s / wr) * cpr + x * wr + s % wr;
        }
    }
    const int64_t g = blk * L + ln;
    const bool act = g < A.lines;
    const int Nz = 2 * M;
    make_twiddles(twM, twN, M);

    double *bd = lds_fft;
    if (DIV) {
        // D = (v_{j+1} - v_j)/dy_j + (w_{k+1} - w_k)/dz at cell (k, j, i); v has
        // Ny+1 faces per plane, w is periodic in k.  Every face value is read
        // by two cells (plain loads, so that the second read finds it cached).
        const int64_t sv = A.lines + A.Nx;          // (Ny+1) Nx
        const int64_t jg = act ? g / A.Nx : 0;
        // reciprocals once a thread (the rows then multiply; FP64 division is
        // a long instruction sequence)
        // u[Nz][Ny][Nx+1] on the x-faces (3-D projection only): face i of cell
        // (j, i) at j (Nx+1) + i in its plane
        constexpr bool has_u = DIV == 2;
        const double idyj = 1.0 / (act ? A.dy[jg] : 1.0), idz = 1.0 / A.dz, idx = has_u ? 1.0 / A.dx : 0.0;
        const int64_t su = A.lines + (A.lines / A.Nx), ug = g + jg;
#pragma unroll
        for (int b0 = 0; b0 < NPT; b0 += NB) {
            double v0[NB], v1[NB], w0[NB], w1[NB], u0[has_u ? NB : 1], u1[has_u ? NB : 1];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int k = tr + (b0 + u) * T;
                v0[u] = v1[u] = w0[u] = w1[u] = 0.0;
                if (has_u) u0[u] = u1[u] = 0.0;
                if (b0 + u < NPT && act && k < Nz) {
                    const int k1 = k + 1 == Nz ? 0 : k + 1;
                    const double *vk = A.v + k * sv + g;
                    v0[u] = vk[0];
                    v1[u] = vk[A.Nx];
                    w0[u] = A.w[k * A.lines + g];
                    w1[u] = A.w[k1 * A.lines + g];
                    if (has_u) {
                        const double *uk = A.u + k * su + ug;
                        u0[u] = uk[0];
                        u1[u] = uk[1];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int k = tr + (b0 + u) * T;
                if (b0 + u < NPT && k < Nz) {
                    double x = 0.0;
                    if (act) {
                        x = (v1[u] - v0[u]) * idyj + (w1[u] - w0[u]) * idz;
                        if (has_u) x = (u1[u] - u0[u]) * idx + x;
                    }
                    bd[((k >> 1) * L + ln) * 2 + (k & 1)] = x;
                }
            }
        }
    } else {
#pragma unroll
        for (int b0 = 0; b0 < NPT; b0 += NB) {
            double x[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int k = tr + (b0 + u) * T;
                x[u] = (b0 + u < NPT && act && k < Nz) ? __builtin_nontemporal_load(A.x + k * A.lines + g) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int k = tr + (b0 + u) * T;
                if (b0 + u < NPT && k < Nz) bd[((k >> 1) * L + ln) * 2 + (k & 1)] = x[u];
            }
        }
    }
    __syncthreads();

    fft_lines<L, MMAX, RSET>(buf, TwFull{twM}, A.S, ln, tr);

    if (!act) return;
    v2d *out = reinterpret_cast<v2d *>(A.xhat);
    for (int k = tr; k <= M / 2; k += T) {
        const cplx zk = buf[(k == 0 ? 0 : k) * L + ln];
        const cplx zm = buf[(k == 0 ? 0 : M - k) * L + ln];
        const cplx e = {0.5 * (zk.re + zm.re), 0.5 * (zk.im - zm.im)};
        const cplx o = {0.5 * (zk.im + zm.im), -0.5 * (zk.re - zm.re)};
        const cplx wo = cmul(twN[k], o);
        const cplx xk = cadd(e, wo);
        const cplx xm = cconj(csub(e, wo));
        __builtin_nontemporal_store(v2d{xk.re, xk.im}, out + (int64_t)k * A.lines + g);
        if (M - k != k) __builtin_nontemporal_store(v2d{xm.re, xm.im}, out + (int64_t)(M - k) * A.lines + g);
    }
}

// Inverse: spectrum rows -> x rows; CORR also corrects w by the spanwise
// gradient of x (the pseudo-pressure): w_k -= (x_k - x_{k-1})/dz, periodic.
// The w rows are loaded before the transform, so that they arrive while it
// runs.
template <int L, int MMAX, bool CORR, int RSET>
__global__ void __launch_bounds__(kFftThreads) k_irfft_z(FftArgs A)
{
    using TL = FftTile<L, MMAX>;
    constexpr int T = TL::T, NPT = TL::NPT, KP = TL::KP;
    extern __shared__ double lds_fft[];
    const int M = A.S.M;
    cplx *buf = reinterpret_cast<cplx *>(lds_fft);
    cplx *twM = buf + (size_t)M * L;
    cplx *twN = twM + M;
    const int ln = threadIdx.x % L, tr = threadIdx.x / L;
    const int64_t g = (int64_t)blockIdx.x * L + ln;
    const bool act = g < A.lines;
    const int Nz = 2 * M;

    // X_k and X_{M-k} of the thread's mode pairs, all loads in flight at once;
    // then the w rows (issued last: loads complete in order, so the spectrum
    // can be used while the w rows are still on their way)
    const v2d *in = reinterpret_cast<const v2d *>(A.xhat_in);
    v2d xa[KP], xb[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const int k = tr + u * T;
        xa[u] = xb[u] = v2d{0.0, 0.0};
        if (act && k <= M / 2) {
            xa[u] = __builtin_nontemporal_load(in + (int64_t)k * A.lines + g);
            xb[u] = __builtin_nontemporal_load(in + (int64_t)(M - k) * A.lines + g);
        }
    }
    double wpre[CORR ? NPT : 1];
    if (CORR) {
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int k = tr + u * T;
            wpre[u] = (act && k < Nz) ? __builtin_nontemporal_load(A.w_io + k * A.lines + g) : 0.0;
        }
    }
    make_twiddles(twM, twN, M);
    __syncthreads();

    // Z_k and Z_{M-k} from X_k and X_{M-k}; stored conjugated, so that the
    // forward passes compute the conjugate of the inverse transform
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const int k = tr + u * T;
        if (k > M / 2) continue;
        cplx a = {xa[u].x, xa[u].y}, b = {xb[u].x, xb[u].y};
        if (k == 0) {
            a.im = 0.0;
            b.im = 0.0;
        }
        const cplx e = {0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};                     // (a + conj b)/2
        const cplx o = cmul({0.5 * (a.re - b.re), 0.5 * (a.im + b.im)}, cconj(twN[k])); // (a - conj b) W^{-k}/2
        const cplx zk = {e.re - o.im, e.im + o.re};                                       // e + i o
        buf[k * L + ln] = cconj(zk);
        if (k != 0 && M - k != k) {
            const cplx zm = {e.re + o.im, -e.im + o.re};                                  // conj e + i conj o
            buf[(M - k) * L + ln] = cconj(zm);
        }
    }
    __syncthreads();

    fft_lines<L, MMAX, RSET>(buf, TwFull{twM}, A.S, ln, tr);

    if (!act) return;
    const double inv_m = 1.0 / M, idz = CORR ? 1.0 / A.dz : 0.0;
    const double *bd = lds_fft;
    // x_{2n} = Re z_n, x_{2n+1} = Im z_n, z = conj(buf)/M
    auto xval = [&](int k) {
        const double t = bd[((k >> 1) * L + ln) * 2 + (k & 1)];
        return (k & 1) ? -t * inv_m : t * inv_m;
    };
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const int k = tr + u * T;
        if (k >= Nz) continue;
        const double x = xval(k);
        __builtin_nontemporal_store(x, A.x_out + k * A.lines + g);
        if (CORR) {
            const double xm = xval(k == 0 ? Nz - 1 : k - 1);
            __builtin_nontemporal_store(wpre[u] - (x - xm) * idz, A.w_io + k * A.lines + g);
        }
    }
}

// Wall-normal gradient correction on the interior y-faces:
// v[k][j][i] -= (phi[k][j][i] - phi[k][j-1][i]) / h_j, h_j = (dy_{j-1} + dy_j)/2,
// j = 1..Ny-1 (the wall faces j = 0 and j = Ny are left as they are).
__global__ void __launch_bounds__(256) k_grad_y(double *v, const double *phi, const double *dy, int Nx, int Ny,
                                                 int nbx)
{
    // workgroup -> (plane row, 256-wide x block); row = k (Ny - 1) + (j - 1)
    const int row = blockIdx.x / nbx;
    const int i = (blockIdx.x - row * nbx) * 256 + threadIdx.x;
    if (i >= Nx) return;
    const int k = row / (Ny - 1);
    const int j = 1 + (row - k * (Ny - 1));
    const double h = 0.5 * (dy[j - 1] + dy[j]);
    const double *p = phi + ((int64_t)k * Ny + j) * Nx + i;
    double *vp = v + ((int64_t)k * (Ny + 1) + j) * Nx + i;
    const double grad = (p[0] - p[-Nx]) / h;
    __builtin_nontemporal_store(__builtin_nontemporal_load(vp) - grad, vp);
}

// Both wall-parallel corrections of the 3-D step from one read of phi: at
// cell (k, j, i), v[k][j][i] -= (phi_j - phi_{j-1})/h_j for j >= 1 and
// u[k][j][i] -= (phi_i - phi_{i-1})/dx for i >= 1 (the neighbours' phi are
// read again from cache); the wall faces j = 0, Ny and i = 0, Nx are left.
// With pp (the time step's pressure, cells like phi) also pp += phi ps.
__global__ void __launch_bounds__(256) k_grad_xy(double *u, double *v, const double *phi, const double *dy, double dx,
                                                  int Nx, int Ny, int nbx, double *pp, double ps)
{
    const int64_t row = blockIdx.x / nbx;                       // k Ny + j
    const int i = (int)(blockIdx.x - row * nbx) * 256 + (int)threadIdx.x;
    if (i >= Nx) return;
    const int64_t k = row / Ny;
    const int j = (int)(row - k * Ny);
    const double *p = phi + row * Nx + i;
    const double pc = p[0];
    if (j >= 1) {
        const double h = 0.5 * (dy[j - 1] + dy[j]);
        double *vp = v + (k * (Ny + 1) + j) * Nx + i;
        __builtin_nontemporal_store(__builtin_nontemporal_load(vp) - (pc - p[-Nx]) / h, vp);
    }
    if (i >= 1) {
        double *up = u + row * (Nx + 1) + i;
        __builtin_nontemporal_store(__builtin_nontemporal_load(up) - (pc - p[-1]) / dx, up);
    }
    if (pp) {
        double *q = pp + row * Nx + i;
        __builtin_nontemporal_store(__builtin_nontemporal_load(q) + pc * ps, q);
    }
}

// ---------------------------------------------------------------------------
// Streamwise cosine transform of complex rows (each row: N values, contiguous):
// X_k = sum_n x_n cos(pi k (2n+1) / (2N)), and its inverse.  Through one
// complex N-point FFT per row: v_n = x_{2n}, v_{N-1-n} = x_{2n+1}, V = DFT(v);
// with A_k = (V_k + conj V_{N-k})/2 and B_k = (V_k - conj V_{N-k})/(2i) (the
// spectra of the real and imaginary parts) and W = exp(-i pi k/(2N)):
// X_k = Re(W A_k) + i Re(W B_k), X_{N-k} = -Im(W A_k) - i Im(W B_k).  The
// inverse forms V_k = conj(W) ((P_k + Q_{N-k}) + i (Q_k - P_{N-k})) from
// P = Re X, Q = Im X (P_N = Q_N = 0), transforms back and unscrambles.
// Rows are transformed in place (a workgroup reads all of its rows before
// it writes them).
template <int L, int NMAX, bool INV>
__global__ void __launch_bounds__(kFftThreads) k_dct_x(DctArgs A)
{
    constexpr int T = kFftThreads / L;
    constexpr int NPT = NMAX / T;
    extern __shared__ double lds_fft[];
    const int N = A.S.M;
    cplx *buf = reinterpret_cast<cplx *>(lds_fft);   // [N + N/16][L] (padded slots)
    auto slot = [](int i) { return fft_slot<true>(i); };
    cplx *lo = buf + (size_t)slot(N) * L;            // W_N^t, t < 64
    cplx *hi = lo + 64;                              // W_N^{64 s}
    const int nhi = (N + 63) / 64;
    cplx *q4 = hi + nhi;                             // W_{4N}^r, r < 4
    const int ln = threadIdx.x % L, tr = threadIdx.x / L;
    const int64_t row = (int64_t)blockIdx.x * L + ln;
    const bool act = row < A.rows;
    v2d *x = reinterpret_cast<v2d *>(A.x) + (act ? row : 0) * A.row_stride;
    for (int t = threadIdx.x; t < 64 + nhi + 4; t += kFftThreads) {
        double sn, cs;
        if (t < 64 + nhi)
            sincospi(2.0 * (t < 64 ? t : 64 * (t - 64)) / N, &sn, &cs);
        else
            sincospi((double)(t - 64 - nhi) / (2 * N), &sn, &cs);
        lo[t] = {cs, -sn};   // hi and q4 follow lo contiguously
    }
    __syncthreads();         // the tables are read before the transform (inverse)
    // exp(-i pi k/(2N)) = W_{4N}^k = W_N^{k/4} W_{4N}^{k mod 4}
    const TwSplit twn{lo, hi};
    auto w4 = [&](int k) { return cmul(twn(k >> 2), q4[k & 3]); };
    if (!INV) {
        v2d xv[NPT];
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int n = tr + u * T;
            xv[u] = (act && n < N) ? __builtin_nontemporal_load(x + n) : v2d{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int n = tr + u * T;
            if (n < N) buf[slot((n & 1) ? N - 1 - (n >> 1) : (n >> 1)) * L + ln] = {xv[u].x, xv[u].y};
        }
    } else {
        constexpr int KP = (NMAX / 2 + 1 + T - 1) / T;
        v2d xa[KP], xb[KP];
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const int k = tr + u * T;
            xa[u] = xb[u] = v2d{0.0, 0.0};
            if (act && k <= N / 2) {
                xa[u] = __builtin_nontemporal_load(x + k);
                if (k > 0) xb[u] = __builtin_nontemporal_load(x + (N - k));
            }
        }
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const int k = tr + u * T;
            if (k > N / 2) continue;
            const cplx wc = cconj(w4(k));                               // conj(W) = exp(+i pi k/(2N))
            const double P = xa[u].x, Q = xa[u].y, Pm = xb[u].x, Qm = xb[u].y;
            const cplx vk = cmul(wc, {P + Qm, Q - Pm});
            buf[slot(k) * L + ln] = cconj(vk);                         // conjugated: inverse by forward passes
            if (k > 0 && N - k != k) {
                // V_{N-k} = conj(W^{N-k})... = i conj(wc) ((P_{N-k} + Q_k) + i (Q_{N-k} - P_k))
                const cplx t = cmul(cconj(wc), {Pm + Q, Qm - P});
                buf[slot(N - k) * L + ln] = cconj(cplx{-t.im, t.re});
            }
        }
    }
    __syncthreads();

    fft_lines<L, NMAX, kRadix8 | kRadix16, TwSplit, true>(buf, TwSplit{lo, hi}, A.S, ln, tr);

    if (!act) return;
    if (!INV) {
        for (int k = tr; k <= N / 2; k += T) {
            const cplx vk = buf[slot(k) * L + ln];
            const cplx vm = buf[slot(k == 0 ? 0 : N - k) * L + ln];
            const cplx a = {0.5 * (vk.re + vm.re), 0.5 * (vk.im - vm.im)};
            const cplx b = {0.5 * (vk.im + vm.im), -0.5 * (vk.re - vm.re)};
            const cplx w = w4(k);
            const cplx wa = cmul(w, a), wb = cmul(w, b);
            __builtin_nontemporal_store(v2d{wa.re, wb.re}, x + k);
            if (k > 0 && N - k != k) __builtin_nontemporal_store(v2d{-wa.im, -wb.im}, x + (N - k));
        }
    } else {
        const double inv_n = 1.0 / N;
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int n = tr + u * T;
            if (n >= N) continue;
            const cplx z = buf[slot((n & 1) ? N - 1 - (n >> 1) : (n >> 1)) * L + ln];
            __builtin_nontemporal_store(v2d{z.re * inv_n, -z.im * inv_n}, x + n);
        }
    }
}

template <int L, int MMAX>
size_t fft_lds_bytes_t(int M)
{
    return sizeof(cplx) * ((size_t)M * L + M + M / 2 + 1);
}

}  // namespace

// Passes of an M-point transform: the radices of `order`, each taken as
// often as it divides what is left (false if M has other prime factors).
static bool make_plan(int M, const int *order, int norder, FftShape &S)
{
    S = FftShape{};
    S.M = M;
    int m = M;
    for (int i = 0; i < norder; ++i)
        while (m % order[i] == 0) {
            if (S.npass == kFftMaxPasses) return false;
            S.radix[S.npass++] = order[i];
            m /= order[i];
        }
    return m == 1;
}

bool fft_shape(int64_t Nz, FftShape &S)
{
    static const int order[4] = {4, 2, 3, 5};
    if (Nz < 2 || (Nz & 1) || Nz / 2 > kFftMaxM) return false;
    return make_plan((int)(Nz / 2), order, 4, S);
}

// Lines per workgroup (measured on MI355X at Nz = 288): 16 for the
// transforms (three workgroups per CU), 32 for the inverse with the w
// correction (its prefetched w rows hold two workgroups per CU anyway);
// TRI_FFT_LINES (8, 16 or 32) overrides where the transform fits that width.
static int fft_lines_per_group(int M, int kind)
{
    const int fit = M <= 144 ? 32 : (M <= 288 ? 16 : 8);
    const char *e = getenv("TRI_FFT_LINES");
    const int want = e ? atoi(e) : 0;
    if ((want == 8 || want == 16 || want == 32) && want <= fit) return want;
    return kind == kFftInverseCorrect ? fit : std::min(fit, 16);
}

// The spanwise transforms use radices 4, 2, 3, 5 (the plan of fft_shape):
// two passes of 16 and 9 at M = 144 measured no faster than four of 4, 4, 3, 3.
template <int L, int MMAX>
static hipError_t launch_fft_t(const FftArgs &A, int kind, hipStream_t s)
{
    const int64_t blocks = (A.lines + L - 1) / L;
    const size_t lds = fft_lds_bytes_t<L, MMAX>(A.S.M);
    const dim3 grid((unsigned)blocks), block(kFftThreads);
    switch (kind) {
    case kFftForward: hipLaunchKernelGGL((k_rfft_z<L, MMAX, 0, 0>), grid, block, lds, s, A); break;
    case kFftDivergence: hipLaunchKernelGGL((k_rfft_z<L, MMAX, 1, 0>), grid, block, lds, s, A); break;
    case kFftDivergence3: hipLaunchKernelGGL((k_rfft_z<L, MMAX, 2, 0>), grid, block, lds, s, A); break;
    case kFftInverse: hipLaunchKernelGGL((k_irfft_z<L, MMAX, false, 0>), grid, block, lds, s, A); break;
    default: hipLaunchKernelGGL((k_irfft_z<L, MMAX, true, 0>), grid, block, lds, s, A); break;
    }
    return hipGetLastError();
}

hipError_t launch_fft(const FftArgs &A, int kind, hipStream_t s)
{
    if (A.lines <= 0) return hipSuccess;
    if ((A.lines + 7) / 8 > 0x7fffffffLL) return hipErrorInvalidValue;
    const int L = fft_lines_per_group(A.S.M, kind);
    if (L == 32) return launch_fft_t<32, 144>(A, kind, s);
    if (L == 16) return A.S.M <= 144 ? launch_fft_t<16, 144>(A, kind, s) : launch_fft_t<16, 288>(A, kind, s);
    return A.S.M <= 144 ? launch_fft_t<8, 144>(A, kind, s) : launch_fft_t<8, kFftMaxM>(A, kind, s);
}

bool dct_shape(int64_t N, FftShape &S)
{
    static const int order[7] = {16, 8, 4, 2, 9, 3, 5};    // 2048 = 16 * 16 * 8: three passes
    if (N < 2 || (N & 1) || N > kDctMaxN) return false;
    return make_plan((int)N, order, 7, S);
}

template <int L, int NMAX>
static hipError_t launch_dct_t(const DctArgs &A, bool inverse, hipStream_t s)
{
    const int64_t blocks = (A.rows + L - 1) / L;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = sizeof(cplx) * ((size_t)(A.S.M + A.S.M / 16) * L + 64 + (A.S.M + 63) / 64 + 4);
    if (inverse)
        hipLaunchKernelGGL((k_dct_x<L, NMAX, true>), dim3((unsigned)blocks), dim3(kFftThreads), lds, s, A);
    else
        hipLaunchKernelGGL((k_dct_x<L, NMAX, false>), dim3((unsigned)blocks), dim3(kFftThreads), lds, s, A);
    return hipGetLastError();
}

hipError_t launch_dct(const DctArgs &A, bool inverse, hipStream_t s)
{
    if (A.rows <= 0) return hipSuccess;
    const char *e = getenv("TRI_DCT_ROWS");
    const int want = e ? atoi(e) : 0;
    if (A.S.M <= 512 && (want == 0 || want == 8)) return launch_dct_t<8, 512>(A, inverse, s);
    // two rows per workgroup (measured on MI355X at N = 2048 and 145 x 256
    // rows: 0.57-0.60 ms against 0.59-0.61 ms with one row); TRI_DCT_ROWS=1
    // selects one row
    if (A.S.M <= 2048 && want == 1) return launch_dct_t<1, 2048>(A, inverse, s);
    if (A.S.M <= 2048) return launch_dct_t<2, 2048>(A, inverse, s);
    return launch_dct_t<1, kDctMaxN>(A, inverse, s);
}

hipError_t launch_grad_xy_pressure(double *u, double *v, const double *phi, const double *dy, double dx, int64_t Nx,
                                   int64_t Ny, int64_t Nz, double *p, double ps, hipStream_t s)
{
    if (Nx < 1 || Ny < 1 || Nz < 1) return hipSuccess;
    const int64_t nbx = (Nx + 255) / 256;
    const int64_t blocks = nbx * Ny * Nz;
    if (blocks > 0x7fffffffLL || Nx > 0x7fffffffLL || Ny > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_grad_xy, dim3((unsigned)blocks), dim3(256), 0, s, u, v, phi, dy, dx, (int)Nx, (int)Ny,
                       (int)nbx, p, ps);
    return hipGetLastError();
}

hipError_t launch_grad_xy(double *u, double *v, const double *phi, const double *dy, double dx, int64_t Nx,
                          int64_t Ny, int64_t Nz, hipStream_t s)
{
    return launch_grad_xy_pressure(u, v, phi, dy, dx, Nx, Ny, Nz, nullptr, 0.0, s);
}

hipError_t launch_grad_y(double *v, const double *phi, const double *dy, int64_t Nx, int64_t Ny, int64_t Nz,
                         hipStream_t s)
{
    if (Ny < 2 || Nx <= 0 || Nz <= 0) return hipSuccess;
    const int64_t nbx = (Nx + 255) / 256;
    const int64_t blocks = nbx * (Ny - 1) * Nz;
    if (blocks > 0x7fffffffLL || Nx > 0x7fffffffLL || Ny > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_grad_y, dim3((unsigned)blocks), dim3(256), 0, s, v, phi, dy, (int)Nx, (int)Ny, (int)nbx);
    return hipGetLastError();
}

}  // namespace tri
