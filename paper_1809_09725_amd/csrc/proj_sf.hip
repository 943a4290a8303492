// Precision form of R_T and R_T*: the basis contraction sum_k Phi[i][k] f_k
// (and its transpose) in BF16 on the matrix cores with FP32 accumulation,
// the projection itself in FP32.
//
// Forward, synthesise-first: for each line (row or column) of slice z the
// states of the line at the Npi half-turns of the workgroup's angle classes
// are formed on MFMA,
//   F[c][pos] = sum_k Phi[i(c)][k] f_k(line, pos),   c = (class slot, half-turn),
// from a BF16 shadow of f (kept beside f~ by the primal update, or converted
// on entry) and Phi split into BF16 hi + lo parts, FP32 accumulate; each ray
// (class, bin) then takes Joseph's two interpolation taps on the frames of
// its class (Sec. 2 eq. Rfwd: the state at time t_i is projected at
// theta_i; the pi-periodicity of Sec. 4 lets every half-turn of a class share
// one ray walk, odd half-turns landing on bin Ns-1-b).
//
// Adjoint: the fold-sum g~(a,z,b,k) = sum_r Phi[r*Ntheta0+a][k] g(r*Ntheta0+a,
// z, b') (Sec. 4) as BF16 MFMA products with FP32 accumulation, then the FP32
// pixel-driven back-projection shared with the plain form.
#include "common.h"
#include "internal.h"

namespace rt {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int ST = 512;        // threads of a synthesise-first workgroup (8 wave64)

// FP32 -> BF16 with round-to-nearest-even (finite inputs).
__device__ inline unsigned short bf16_rne(float x)
{
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

struct SfEpi {
    float *out;           // g (EPI_G) or h1 (EPI_PROX); with line parts: partial sums
    const float *gdata;   // measured sinogram (EPI_PROX)
    double *part;         // per-workgroup FP64 sum of (R f~ - g)^2, or NULL
    size_t pstride;       // line parts: floats between the parts' partial sums
    float sigma;
    int prox, n0, Npi;
};

// Forward, synthesise-first.  Workgroup: slice z, a group of A classes of one
// walk direction, bins [bt*BT, bt*BT + BT), and part lp of the NLP parts of
// the slice's lines (NLP > 1: the ray sums over those lines are stored at
// E.out + lp * E.pstride for k_sf_finish).  Consecutive workgroups take the
// class groups of one part, so the part's BF16 lines are read while they are
// still cached.  Thread t owns the rays (slot j, bin bt*BT + t') for the A
// slots, t' being t reordered within its wave by slot j's lane map.  NPP:
// frame columns per class (Npi rounded up to 4, the padding columns are
// zero); KB: MFMA k-steps of 16 channels.
//
// The frames F[c][pos] = sum_k Phi[i(c)][k] f_k(pos) of a chunk of PCH
// positions are one v_mfma_f32_32x32x16_bf16 product per 32-position tile:
// A = Phi rows of the 32 frame columns (hi and lo BF16 parts), B = the BF16
// shadow of f.  They land in LDS position-major, row 1 + pos - c0 holding the
// A*NPP frames of position pos, so that a ray's tap at one position is NPP/4
// 16-byte reads, the access of the plain form's staged lines.
// The bin offset thread tid takes for class a: its own, reordered within its
// wave's block of 64 bins by the class's lane map (the 16-lane tap reads at
// positions 1/|c| apart then spread over the LDS bank groups; the row stride
// CS is an odd number of 16-byte groups).
__device__ inline int sf_bin(int tid, int a, const unsigned char *__restrict__ lperm)
{
    return a >= 0 ? (tid & ~63) | (int)lperm[a * 64 + (tid & 63)] : tid;
}

template <int NPP, int KB, int AS, int UB, int DS>
__global__ __launch_bounds__(ST) void k_project_sf(
    const __bf16 *__restrict__ f16, const float *__restrict__ phi, const int *__restrict__ gcls,
    const int *__restrict__ gwalk, const unsigned char *__restrict__ lperm, const double *__restrict__ ccos,
    const double *__restrict__ csin, int N, int Nz, int Ns, int K, int A, int ngroups, int BT,
    int nbt, int PCH, int CS, int NLP, unsigned nblocks, SfEpi E)
{
    constexpr int KP = 16 * KB;
    constexpr int R = AS * UB;      // rays per thread: slot rho / UB, bin sf_bin(tid) + ST * (rho % UB)
    extern __shared__ float fr[];   // [PCH + 2][CS]; rows 0 and PCH + 1 stay zero
    __shared__ double sh[ST / 64];
    unsigned lid = xcd_remap(blockIdx.x, nblocks);
    const int bt = lid % nbt;
    lid /= nbt;
    const int grp = lid % ngroups;
    lid /= ngroups;
    const int lp = lid % NLP;
    const int z = lid / NLP;
    const int lbeg = (int)((long)lp * N / NLP), lend = (int)((long)(lp + 1) * N / NLP);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int walk = gwalk[grp];
    const int Npi = E.Npi;
    const int CW = A * NPP;        // frame columns in use
    const double hN = 0.5 * (double)(N - 1), hS = 0.5 * (double)(Ns - 1);

    // ---- rays of this thread
    double base[R], slope[R];
    float invc[R];
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
        const int j = rho / UB;
        const int a = j < A ? gcls[grp * A + j] : -1;
        const int bi = sf_bin(tid, a, lperm) + ST * (rho % UB), b = bt * BT + bi;
        base[rho] = -1.0e9;   // far outside: never tapped
        slope[rho] = 0.0;
        invc[rho] = 0.f;
        if (a >= 0 && bi < BT && b < Ns) {
            const double cs = ccos[a], sn = csin[a], sb = (double)b - hS;
            if (walk == 0) {
                base[rho] = sb / cs + hN;
                slope[rho] = -sn / cs;
                invc[rho] = (float)(1.0 / fabs(cs));
            } else {
                base[rho] = sb / sn + hN;
                slope[rho] = -cs / sn;
                invc[rho] = (float)(1.0 / fabs(sn));
            }
        }
    }
    float acc[R][NPP];
#pragma unroll
    for (int rho = 0; rho < R; ++rho)
#pragma unroll
        for (int r = 0; r < NPP; ++r) acc[rho][r] = 0.f;

    // ---- MFMA A operand: Phi[i(c)][k] of frame column c = lane % 32 (slot
    // c / NPP, half-turn c % NPP), channels kb*16 + 8*(lane/32) + 0..7
    v8bf ahi[KB], alo[KB];
    {
        const int c = lane & 31, slot = c / NPP, r = c % NPP;
        const int a = (slot < A && r < Npi) ? gcls[grp * A + slot] : -1;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int k = kb * 16 + 8 * (lane >> 5) + q;
                const float v = (a >= 0 && k < K) ? phi[(size_t)(r * E.n0 + a) * K + k] : 0.f;
                const __bf16 h = (__bf16)v;
                ahi[kb][q] = h;
                alo[kb][q] = (__bf16)(v - (float)h);
            }
    }

    for (int e = tid; e < 2 * CS; e += ST) fr[e < CS ? e : (PCH + 1) * CS + (e - CS)] = 0.f;

    const __bf16 *fz = f16 + (size_t)z * N * N * KP;
    const size_t lstep = walk == 0 ? (size_t)N * KP : (size_t)KP;
    const size_t pstep = walk == 0 ? (size_t)KP : (size_t)N * KP;
    const int nch = (N + PCH - 1) / PCH;
    const int nsteps = (lend - lbeg) * nch;   // (line, chunk) steps of this part

    // B operand of one step for the wave's position tiles wave and wave + 8:
    // lane holds position c0 + tile*32 + lane%32, channels kb*16 + 8*(lane/32) + 0..7
    v8bf raw[2][KB];
    auto load_step = [&](int st) {
        const int l = lbeg + st / nch, c0 = (st % nch) * PCH;
        const __bf16 *src = fz + (size_t)l * lstep + 8 * (lane >> 5);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = wave + 8 * h;
            const int pos = c0 + t * 32 + (lane & 31);
            const bool in = t * 32 < PCH && pos < N;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                raw[h][kb] = in ? *(const v8bf *)(src + (size_t)pos * pstep + kb * 16) : v8bf{};
        }
    };
    // DS > 0: the B operand goes global -> LDS directly, DS - 1 steps ahead,
    // into a ring of DS stages private to the wave (NI copies of 64 x 16
    // bytes per step).  The copies are issued from inline assembly, so the
    // compiler does not treat them as LDS stores and adds no wait for them
    // before the frame and tap reads; each step waits for its own copies with
    // an explicit vmcnt.  Every copy reads a valid address (positions clamped
    // to the slice, steps clamped to the last one), so the count per step is
    // fixed; lanes outside the slice or the chunk are zeroed after the read.
    constexpr int NI = 2 * KB;
    char *wring = (char *)(fr + (size_t)(PCH + 2) * CS) + (size_t)wave * (DS > 0 ? DS : 1) * NI * 1024;
    auto issue_step = [&](int st) {
        const int sc = min(st, nsteps - 1);
        const int l = lbeg + sc / nch, c0 = (sc % nch) * PCH;
        const __bf16 *src = fz + (size_t)l * lstep + 8 * (lane >> 5);
        char *dst = wring + (size_t)(st % (DS > 0 ? DS : 1)) * NI * 1024;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = wave + 8 * h;
            const int pos = min(c0 + t * 32 + (lane & 31), N - 1);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const __bf16 *ga = src + (size_t)pos * pstep + kb * 16;
                const unsigned la = (unsigned)(size_t)(dst + (h * KB + kb) * 1024);
                // the LDS destination goes in m0, bound as an input operand
                asm volatile("global_load_lds_dwordx4 %0, off"
                             :: "v"(ga), "{m0}"(__builtin_amdgcn_readfirstlane(la)) : "memory");
            }
        }
    };
    if constexpr (DS > 0) {
        if (nsteps > 0)
            for (int d = 0; d < DS - 1; ++d) issue_step(d);
    } else {
        if (nsteps > 0) load_step(0);
    }

    // Ray positions in 32.32 fixed point, as in the plain projector: u at
    // line lbeg from FP64 once, then one exact integer add of the slope per
    // line (the position carries the rounding of its start and of l s alone,
    // below 2^-32 (1 + l)).  A ray outside the tile sits at -1e6.
    long long U[R], Sl[R];
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
        const double u0 = fmin(fmax(fma((double)lbeg - hN, slope[rho], base[rho]), -1.0e6), 1.0e6);
        U[rho] = (long long)llrint(u0 * 4294967296.0);
        Sl[rho] = (long long)llrint(slope[rho] * 4294967296.0);
    }
    int q0[R];
    float w0[R], w1[R];
    for (int st = 0; st < nsteps; ++st) {
        const int c0 = (st % nch) * PCH;
        if (c0 == 0) {   // ray positions on this step's line
#pragma unroll
            for (int rho = 0; rho < R; ++rho) {
                const int q = (int)(U[rho] >> 32);
                const float frc = (float)(unsigned)U[rho] * 2.3283064365386963e-10f;
                U[rho] += Sl[rho];
                const bool in = (unsigned)(q + 1) <= (unsigned)N;
                q0[rho] = in ? q : -(1 << 28);
                w1[rho] = in ? frc * invc[rho] : 0.f;
                w0[rho] = in ? (1.f - frc) * invc[rho] : 0.f;
            }
        }
        v8bf bop[2][KB];
        if constexpr (DS > 0) {
            issue_step(st + DS - 1);   // into the stage step st - 1 has finished with
            asm volatile("s_waitcnt vmcnt(%0)" :: "n"(NI * (DS - 1)) : "memory");
            const char *src = wring + (size_t)(st % DS) * NI * 1024 + lane * 16;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = wave + 8 * h;
                const bool in = t * 32 < PCH && c0 + t * 32 + (lane & 31) < N;
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const v8bf x = *(const v8bf *)(src + (h * KB + kb) * 1024);
                    bop[h][kb] = in ? x : v8bf{};
                }
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) bop[h][kb] = raw[h][kb];
            if (st + 1 < nsteps) load_step(st + 1);
        }
        v16f d0 = {}, d1 = {};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            d0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[kb], bop[0][kb], d0, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[kb], bop[1][kb], d1, 0, 0, 0);
            d0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[kb], bop[0][kb], d0, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[kb], bop[1][kb], d1, 0, 0, 0);
        }
        __syncthreads();   // the previous step's taps are done with the frames
        // D[c][pos]: lane holds position lane%32 of its tile, columns 8g + 4(lane/32) + 0..3
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = wave + 8 * h;
            if (t * 32 >= PCH) continue;
            const v16f &d = h ? d1 : d0;
            float *row = fr + (1 + t * 32 + (lane & 31)) * CS + 4 * (lane >> 5);
#pragma unroll
            for (int g = 0; g < 4; ++g)
                if (8 * g + 4 * (lane >> 5) < CW)
                    *(float4 *)(row + 8 * g) = make_float4(d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]);
        }
        __syncthreads();
        // taps of the rays whose positions fall in this chunk
#pragma unroll
        for (int rho = 0; rho < R; ++rho) {
            const int q = q0[rho] - c0;
            const bool t0 = q >= 0 && q < PCH;
            const bool t1 = q >= -1 && q < PCH - 1;
            if (!(t0 || t1)) continue;
            const float a0 = t0 ? w0[rho] : 0.f, a1 = t1 ? w1[rho] : 0.f;
            const float *F0 = fr + (q + 1) * CS + (rho / UB) * NPP;
#pragma unroll
            for (int m = 0; m < NPP / 4; ++m) {
                const float4 x0 = *(const float4 *)(F0 + 4 * m);
                const float4 x1 = *(const float4 *)(F0 + CS + 4 * m);
                acc[rho][4 * m + 0] = fmaf(a1, x1.x, fmaf(a0, x0.x, acc[rho][4 * m + 0]));
                acc[rho][4 * m + 1] = fmaf(a1, x1.y, fmaf(a0, x0.y, acc[rho][4 * m + 1]));
                acc[rho][4 * m + 2] = fmaf(a1, x1.z, fmaf(a0, x0.z, acc[rho][4 * m + 2]));
                acc[rho][4 * m + 3] = fmaf(a1, x1.w, fmaf(a0, x0.w, acc[rho][4 * m + 3]));
            }
        }
    }

    if constexpr (DS > 0) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the last copies landed

    // ---- epilogue: every half-turn r of class a lands on bin b (even r) or Ns-1-b (odd r)
    double d2 = 0.0;
    const float inv1s = 1.f / (1.f + E.sigma);
    // out and gdata do not overlap: the loads of all half-turns may be issued
    // ahead of the stores
    const float *__restrict__ gd = E.gdata;
    float *__restrict__ out = E.out;
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
        const int j = rho / UB;
        const int a = j < A ? gcls[grp * A + j] : -1;
        const int bi = sf_bin(tid, a, lperm) + ST * (rho % UB), b = bt * BT + bi;
        if (a < 0 || bi >= BT || b >= Ns) continue;
#pragma unroll
        for (int r = 0; r < NPP; ++r) {
            if (r >= Npi) continue;
            const int i = r * E.n0 + a;
            const int bo = (r & 1) ? Ns - 1 - b : b;
            const size_t o = ((size_t)i * Nz + z) * Ns + bo;
            const float v = acc[rho][r];
            if (!E.prox) {
                out[o + lp * E.pstride] = v;
            } else {
                const float d = v - gd[o];
                d2 += (double)d * (double)d;
                out[o] = (out[o] + E.sigma * d) * inv1s;
            }
        }
    }
    if (E.part) {
        const double sum = block_sum(d2, sh);
        if (tid == 0) E.part[blockIdx.x] = sum;
    }
}

// The line parts' partial ray sums added in part order, then stored as g or
// taken into the h1 prox of Fig. 2 step 3 with the FP64 partial sums of
// (R f~ - g)^2; rows grid-strided over a fixed number of workgroups.
__global__ __launch_bounds__(NT) void k_sf_finish(const float *__restrict__ psf, int NLP,
                                                  size_t ng, float *__restrict__ out,
                                                  const float *__restrict__ gdata, int prox,
                                                  float sigma, double *__restrict__ part)
{
    __shared__ double sh[NT / 64];
    double d2 = 0.0;
    const float inv1s = 1.f / (1.f + sigma);
    for (size_t o = (size_t)blockIdx.x * NT + threadIdx.x; o < ng; o += (size_t)gridDim.x * NT) {
        float v = psf[o];
        for (int lp = 1; lp < NLP; ++lp) v += psf[(size_t)lp * ng + o];
        if (!prox) {
            out[o] = v;
        } else {
            const float d = v - gdata[o];
            d2 += (double)d * (double)d;
            out[o] = (out[o] + sigma * d) * inv1s;
        }
    }
    if (part) {
        const double s = block_sum(d2, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    }
}

unsigned sf_finish_blocks(const rt_geom &G)
{
    const size_t ng = ng_of(G);
    return (unsigned)std::max<size_t>(1, std::min<size_t>((ng + NT - 1) / NT, 8192));
}

// BF16 shadow of f: [Nz][N][N][K] FP32 -> [Nz][N][N][KP] BF16 (round to
// nearest even), channels K..KP-1 zero.  One thread per 8 output channels.
__global__ __launch_bounds__(NT) void k_to_bf16(const float *__restrict__ f,
                                                __bf16 *__restrict__ out, size_t nvox, int K,
                                                int KP)
{
    const int n8 = KP / 8;
    const size_t total = nvox * n8;
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < total;
         e += (size_t)gridDim.x * NT) {
        const size_t v = e / n8;
        const int k0 = (int)(e % n8) * 8;
        const float *src = f + v * K;
        v8bf o;
#pragma unroll
        for (int q = 0; q < 8; ++q) o[q] = (__bf16)(k0 + q < K ? src[k0 + q] : 0.f);
        *(v8bf *)(out + v * KP + k0) = o;
    }
}

// Fold-sum on MFMA (v_mfma_f32_16x16x16 bf16): per (class a, slice z) the
// product [Ns bins x Npi half-turns] x [Npi x K], half-turns padded to a
// multiple of 16.  One wave per 16-bin x 16-channel tile.
// A: lane holds bins row = lane%16, half-turns 4*(lane/16) + 0..3 of the
// current 16-chunk; B: Phi rows of those half-turns, channel lane%16;
// C: bins 4*(lane/16) + 0..3, channel lane%16.
// Both operands are split into BF16 hi + lo parts and the three products
// hi*hi + hi*lo + lo*hi are accumulated in FP32 (the lo*lo term is below
// 2^-16 of the product): the sinogram fed to the adjoint is the dual h1 of
// the data term, whose rounding to a single BF16 would put a 2^-9 relative
// error straight into the primal update when few half-turns and classes
// average it.  The fold is bound by its HBM traffic, so the two extra
// products cost nothing measurable.
__global__ __launch_bounds__(NT) void k_fold_mfma(const float *__restrict__ g,
                                                  const float *__restrict__ phi,
                                                  float *__restrict__ gt, int Nz, int Ns, int K,
                                                  int n0, int Npi)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nbt = (Ns + 15) / 16, nkt = (K + 15) / 16;
    const long tiles = (long)n0 * Nz * nbt * nkt;
    for (long t = (long)blockIdx.x * (NT / 64) + wave; t < tiles; t += (long)gridDim.x * (NT / 64)) {
        long u = t;
        const int kt = (int)(u % nkt);
        u /= nkt;
        const int btile = (int)(u % nbt);
        u /= nbt;
        const int z = (int)(u % Nz);
        const int a = (int)(u / Nz);
        const int bin = btile * 16 + (lane & 15);
        const int kcol = kt * 16 + (lane & 15);
        v4f cacc = {0.f, 0.f, 0.f, 0.f};
        for (int r0 = 0; r0 < Npi; r0 += 16) {
            v4s ah, al, bh, bl;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + 4 * (lane >> 4) + q;
                float gv = 0.f, pv = 0.f;
                if (r < Npi) {
                    const int i = r * n0 + a;
                    if (bin < Ns) gv = g[((size_t)i * Nz + z) * Ns + ((r & 1) ? Ns - 1 - bin : bin)];
                    if (kcol < K) pv = phi[(size_t)i * K + kcol];
                }
                const unsigned short gh = bf16_rne(gv);
                ah[q] = (short)gh;
                al[q] = (short)bf16_rne(gv - bf16_val(gh));
                const unsigned short h = bf16_rne(pv);
                bh[q] = (short)h;
                bl[q] = (short)bf16_rne(pv - bf16_val(h));
            }
            cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, cacc, 0, 0, 0);
            cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, cacc, 0, 0, 0);
            cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, cacc, 0, 0, 0);
        }
        if (kcol < K) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int bo = btile * 16 + 4 * (lane >> 4) + q;
                if (bo < Ns) gt[(((size_t)a * Nz + z) * Ns + bo) * K + kcol] = cacc[q];
            }
        }
    }
}

template <int NPP, int KB, int AS, int UB, int DS>
static int launch_sf_d(const Plan &p, const SfEpi &E, hipStream_t s, unsigned nb)
{
    const rt_geom &G = p.g;
    const SfCfg &C = p.sf;
    auto kern = k_project_sf<NPP, KB, AS, UB, DS>;
    if (C.lds > 64 * 1024)
        RT_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)C.lds));
    KTimer kt("k_project_sf", s);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(ST), C.lds, s, (const __bf16 *)p.d_f16, p.d_phi,
                       p.d_gcls_sf, p.d_gwalk_sf, p.d_lperm, p.d_ccos, p.d_csin, G.N, G.Nz, G.Ns, G.K, C.A,
                       C.ngroups, C.BT, C.nbt, C.PCH, C.CS, C.NLP, nb, E);
    kt.stop();
    return RT_OK;
}

// the staged B operand is planned for KB = 2 only
template <int NPP, int KB, int AS, int UB>
static int launch_sf_t(const Plan &p, const SfEpi &E, hipStream_t s, unsigned nb)
{
    if constexpr (KB == 2) {
        if (p.sf.DS == 3) return launch_sf_d<NPP, KB, AS, UB, 3>(p, E, s, nb);
    }
    return launch_sf_d<NPP, KB, AS, UB, 0>(p, E, s, nb);
}

// AS slots for one bin per thread; UB bins per thread take AS / UB slots
// the slot count sf_slots gives: at most 96 ray sums and 8 rays per thread
// (64 and 4 when K > 32)
constexpr int acc_cap(int kb) { return kb >= 3 ? 64 : 96; }
constexpr int fit_slots(int as, int ub, int npp, int kb)
{
    return (as > 1 && (as * ub * npp > acc_cap(kb) || as * ub > (kb >= 3 ? 4 : 8)))
               ? fit_slots(as - 1, ub, npp, kb) : as;
}

template <int NPP, int KB, int AS>
static int launch_sf_u(const Plan &p, const SfEpi &E, hipStream_t s, unsigned nb)
{
    constexpr int AS2 = fit_slots(AS, 2, NPP, KB), AS4 = fit_slots(AS, 4, NPP, KB);
    switch (p.sf.UB) {
    case 1: return launch_sf_t<NPP, KB, fit_slots(AS, 1, NPP, KB), 1>(p, E, s, nb);
    case 2: return launch_sf_t<NPP, KB, AS2, 2>(p, E, s, nb);
    default:
        // the plan keeps UB * slots * NPP within acc_cap accumulators per thread
        if constexpr (4 * AS4 * NPP <= acc_cap(KB)) {
            return launch_sf_t<NPP, KB, AS4, 4>(p, E, s, nb);
        } else {
            return fail(RT_E_SHAPE, "no synthesise-first kernel for NPP=%d with 4 bins per thread", NPP);
        }
    }
}

template <int NPP, int AS>
static int launch_sf_k(const Plan &p, const SfEpi &E, hipStream_t s, unsigned nb)
{
    switch (p.sf.KP / 16) {
    case 1: return launch_sf_u<NPP, 1, AS>(p, E, s, nb);
    case 2: return launch_sf_u<NPP, 2, AS>(p, E, s, nb);
    case 3: return launch_sf_u<NPP, 3, AS>(p, E, s, nb);
    default: return launch_sf_u<NPP, 4, AS>(p, E, s, nb);
    }
}

}  // namespace

unsigned sf_blocks(const Plan &p)
{
    return (unsigned)p.g.Nz * p.sf.ngroups * p.sf.nbt * p.sf.NLP;
}

// FP64 partials of the forward's h1 prox: one per projection workgroup, or one
// per k_sf_finish workgroup when the lines come in parts
unsigned sf_partials(const Plan &p) { return p.sf.NLP > 1 ? sf_finish_blocks(p.g) : sf_blocks(p); }

int sf_slots(int npp, int ub, int kb)
{
    int as = npp <= 8 ? 4 : npp <= 16 ? 2 : 1;
    while (as > 1 && (as * ub * npp > (kb >= 3 ? 64 : 96) || as * ub > (kb >= 3 ? 4 : 8))) --as;
    return as;
}

int launch_to_bf16(const Plan &p, const float *f, hipStream_t s)
{
    const rt_geom &G = p.g;
    const size_t nvox = (size_t)G.Nz * G.N * G.N;
    if (nvox == 0) return RT_OK;
    const size_t total = nvox * (p.sf.KP / 8);
    const unsigned nb = (unsigned)std::min<size_t>((total + NT - 1) / NT, 16384);
    KTimer kt("k_to_bf16", s);
    hipLaunchKernelGGL(k_to_bf16, dim3(nb), dim3(NT), 0, s, f, (__bf16 *)p.d_f16, nvox, G.K,
                       p.sf.KP);
    kt.stop();
    RT_HIP(hipGetLastError());
    ++p.shadow_gen;
    return RT_OK;
}

int launch_forward_sf16(const Plan &p, float *g, int mode, const float *gdata, float *h1,
                        float sigma, double *part, hipStream_t s)
{
    const rt_geom &G = p.g;
    if (G.Nz == 0) return RT_OK;
    SfEpi E{};
    float *dst = mode == CONTRACT_STORE ? g : h1;
    const bool parts = p.sf.NLP > 1;
    E.out = parts ? p.d_psf : dst;
    E.gdata = gdata;
    E.part = parts ? nullptr : part;
    E.pstride = parts ? ng_of(G) : 0;
    E.sigma = sigma;
    E.prox = !parts && mode == CONTRACT_PROX;
    E.n0 = p.n0;
    E.Npi = G.Npi;
    const unsigned nb = sf_blocks(p);
    int rc;
    switch (p.sf.NPP) {
    case 4: rc = launch_sf_k<4, 4>(p, E, s, nb); break;
    case 8: rc = launch_sf_k<8, 4>(p, E, s, nb); break;
    case 12: rc = launch_sf_k<12, 2>(p, E, s, nb); break;
    case 16: rc = launch_sf_k<16, 2>(p, E, s, nb); break;
    case 20: rc = launch_sf_k<20, 1>(p, E, s, nb); break;
    case 24: rc = launch_sf_k<24, 1>(p, E, s, nb); break;
    case 28: rc = launch_sf_k<28, 1>(p, E, s, nb); break;
    default: rc = launch_sf_k<32, 1>(p, E, s, nb); break;
    }
    if (rc) return rc;
    RT_HIP(hipGetLastError());
    if (parts) {
        KTimer kt("k_sf_finish", s);
        hipLaunchKernelGGL(k_sf_finish, dim3(sf_finish_blocks(G)), dim3(NT), 0, s, p.d_psf,
                           p.sf.NLP, ng_of(G), dst, gdata, mode == CONTRACT_PROX ? 1 : 0, sigma,
                           part);
        kt.stop();
        RT_HIP(hipGetLastError());
    }
    return RT_OK;
}

int launch_forward_sf(const Plan &p, const float *f, float *g, int mode, const float *gdata,
                      float *h1, float sigma, double *part, hipStream_t s)
{
    if (p.g.Nz == 0) return RT_OK;
    int rc = launch_to_bf16(p, f, s);
    if (rc) return rc;
    return launch_forward_sf16(p, g, mode, gdata, h1, sigma, part, s);
}

int launch_fold_mfma(const Plan &p, const float *g, hipStream_t s)
{
    const rt_geom &G = p.g;
    if (G.Nz == 0) return RT_OK;
    const long tiles = (long)p.n0 * G.Nz * ((G.Ns + 15) / 16) * ((G.K + 15) / 16);
    const unsigned nb = (unsigned)std::max<long>(1, std::min<long>((tiles + 3) / 4, 16384));
    KTimer kt("k_fold_mfma", s);
    hipLaunchKernelGGL(k_fold_mfma, dim3(nb), dim3(NT), 0, s, g, p.d_phi, p.d_scr, G.Nz, G.Ns,
                       G.K, p.n0, G.Npi);
    kt.stop();
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rt
