// Precision form of R_T and R_T*: the basis contraction sum_k Phi[i][k] f_k
// (and its transpose) in BF16 on the matrix cores with FP32 accumulation,
// the projection itself in FP32.
//
// Forward, synthesise-first: for each staged line (row or column) of slice z
// the states of the line at the Npi half-turns of the workgroup's angle
// classes are formed on MFMA,
//   F[c][pos] = sum_k f_k(line, pos) Phi[i(c)][k],   c = (class slot, half-turn),
// with f_k rounded to BF16 and Phi split into BF16 hi + lo, FP32 accumulate;
// each ray (class, bin) then takes Joseph's two interpolation taps on the
// Npi frame lines of its class (Sec. 2 eq. Rfwd: the state at time t_i is
// projected at theta_i; the pi-periodicity of Sec. 4 lets every half-turn of
// a class share one ray walk, odd half-turns landing on bin Ns-1-b).
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

constexpr int ST = 512;        // threads of a synthesise-first workgroup (8 wave64)
constexpr int SF_COLS = 32;    // frame columns per workgroup: one 32-wide MFMA tile
constexpr int SF_PAD = 4;      // LDS slots before position 0 of a chunk (16-byte alignment)

// FP32 -> BF16 with round-to-nearest-even (finite inputs).
__device__ inline unsigned short bf16_rne(float x)
{
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

struct SfEpi {
    float *out;           // g (EPI_G) or h1 (EPI_PROX)
    const float *gdata;   // measured sinogram (EPI_PROX)
    double *part;         // per-workgroup FP64 sum of (R f~ - g)^2, or NULL
    float sigma;
    int prox, n0, Npi;
};

// Workgroup: slice z, a group of A classes of one walk direction, bins
// [bt*BT, bt*BT + BT).  Thread t owns the rays (slot j, bin bt*BT + t) for
// the A slots.  NPM: accumulators per ray (>= Npi).  KB: K / 8 (MFMA k-steps).
template <int NPM, int KB, int AS>
__global__ __launch_bounds__(ST) void k_project_sf(
    const float *__restrict__ f, const float *__restrict__ phi, const int *__restrict__ gcls,
    const int *__restrict__ gwalk, const double *__restrict__ ccos,
    const double *__restrict__ csin, int N, int Nz, int Ns, int K, int A, int ngroups, int BT,
    int nbt, int PCH, int cstride, unsigned nblocks, SfEpi E)
{
    extern __shared__ float fr[];   // [SF_COLS][cstride]: frame c at slot SF_PAD + pos - c0
    __shared__ double sh[ST / 64];
    unsigned lid = xcd_remap(blockIdx.x, nblocks);
    const int bt = lid % nbt;
    lid /= nbt;
    const int grp = lid % ngroups;
    const int z = lid / ngroups;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int walk = gwalk[grp];
    const int Npi = E.Npi;
    const double hN = 0.5 * (double)(N - 1), hS = 0.5 * (double)(Ns - 1);

    // ---- rays of this thread
    const int b = bt * BT + tid;
    double base[AS], slope[AS];
    float invc[AS];
#pragma unroll
    for (int j = 0; j < AS; ++j) {
        const int a = j < A ? gcls[grp * A + j] : -1;
        base[j] = -1.0e9;   // far outside: both taps get weight 0
        slope[j] = 0.0;
        invc[j] = 0.f;
        if (a >= 0 && tid < BT && b < Ns) {
            const double cs = ccos[a], sn = csin[a], sb = (double)b - hS;
            if (walk == 0) {
                base[j] = sb / cs + hN;
                slope[j] = -sn / cs;
                invc[j] = (float)(1.0 / fabs(cs));
            } else {
                base[j] = sb / sn + hN;
                slope[j] = -cs / sn;
                invc[j] = (float)(1.0 / fabs(sn));
            }
        }
    }
    float acc[AS][NPM];
#pragma unroll
    for (int j = 0; j < AS; ++j)
#pragma unroll
        for (int r = 0; r < NPM; ++r) acc[j][r] = 0.f;

    // ---- MFMA B operand: Phi^T[k][c] for the 32 frame columns, hi and lo parts.
    // lane holds column c = lane % 32, channels kb*8 + 4*(lane/32) + 0..3.
    v4s bhi[KB], blo[KB];
    {
        const int c = lane & 31, slot = c / Npi, r = c % Npi;
        const int a = (slot < A) ? gcls[grp * A + slot] : -1;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = kb * 8 + 4 * (lane >> 5) + q;
                float v = 0.f;
                if (a >= 0 && k < K) v = phi[(size_t)(r * E.n0 + a) * K + k];
                const unsigned short h = bf16_rne(v);
                bhi[kb][q] = (short)h;
                blo[kb][q] = (short)bf16_rne(v - bf16_val(h));
            }
        }
    }

    // zero the pad slots (never written by the frame stores)
    for (int e = tid; e < SF_COLS * 2 * SF_PAD; e += ST) {
        const int c = e / (2 * SF_PAD), s = e % (2 * SF_PAD);
        fr[c * cstride + (s < SF_PAD ? s : SF_PAD + PCH + (s - SF_PAD))] = 0.f;
    }

    const size_t zoff = (size_t)z * N * N * K;
    const size_t lstep = walk == 0 ? (size_t)N * K : (size_t)K;
    const size_t pstep = walk == 0 ? (size_t)K : (size_t)N * K;
    const int nch = (N + PCH - 1) / PCH;
    const int nsteps = N * nch;          // (line, chunk) steps

    // A operand of one step for the wave's two row tiles (wave, wave + 8):
    // lane holds position c0 + tile*32 + lane%32, channels kb*8 + 4*(lane/32) + 0..3.
    float4 raw[2][KB];
    auto load_step = [&](int st) {
        const int l = st / nch, c0 = (st % nch) * PCH;
        const float *src = f + zoff + (size_t)l * lstep;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = wave + 8 * h;
            const int pos = c0 + t * 32 + (lane & 31);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const int k = kb * 8 + 4 * (lane >> 5);
                float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t * 32 < PCH && pos < N) {
                    const float *p = src + (size_t)pos * pstep + k;
                    if ((K & 3) == 0 && k + 3 < K) {
                        x = *(const float4 *)p;
                    } else {
                        x.x = k < K ? p[0] : 0.f;
                        x.y = k + 1 < K ? p[1] : 0.f;
                        x.z = k + 2 < K ? p[2] : 0.f;
                        x.w = k + 3 < K ? p[3] : 0.f;
                    }
                }
                raw[h][kb] = x;
            }
        }
    };
    load_step(0);

    int q0[AS];
    float w0[AS], w1[AS];
    for (int st = 0; st < nsteps; ++st) {
        const int l = st / nch, ch = st % nch, c0 = ch * PCH;
        if (ch == 0) {   // ray positions on line l
            const double lc = (double)l - hN;
#pragma unroll
            for (int j = 0; j < AS; ++j) {
                const double u = fma(lc, slope[j], base[j]);
                const double fl = floor(u);
                const int q = (int)fl;
                const float frc = (float)(u - fl);
                const bool in = (unsigned)(q + 1) <= (unsigned)N;
                q0[j] = in ? q : -2;
                w1[j] = in ? frc * invc[j] : 0.f;
                w0[j] = in ? (1.f - frc) * invc[j] : 0.f;
            }
        }
        // this step's A operands to BF16, then start the next step's loads
        v4s av[2][KB];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                av[h][kb][0] = (short)bf16_rne(raw[h][kb].x);
                av[h][kb][1] = (short)bf16_rne(raw[h][kb].y);
                av[h][kb][2] = (short)bf16_rne(raw[h][kb].z);
                av[h][kb][3] = (short)bf16_rne(raw[h][kb].w);
            }
        if (st + 1 < nsteps) load_step(st + 1);
        // frames of the two tiles on MFMA (two independent accumulators)
        v16f c0acc = {}, c1acc = {};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            c0acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av[0][kb], bhi[kb], c0acc, 0, 0, 0);
            c1acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av[1][kb], bhi[kb], c1acc, 0, 0, 0);
            c0acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av[0][kb], blo[kb], c0acc, 0, 0, 0);
            c1acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av[1][kb], blo[kb], c1acc, 0, 0, 0);
        }
        __syncthreads();   // the previous step's taps are done with the frame buffer
        // D[row][col]: lane holds column lane%32, rows 8*(v/4) + 4*(lane/32) + v%4
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = wave + 8 * h;
            if (t * 32 >= PCH) continue;
            const v16f &cc = h ? c1acc : c0acc;
            float *Fc = fr + (lane & 31) * cstride + SF_PAD + t * 32 + 4 * (lane >> 5);
#pragma unroll
            for (int g4 = 0; g4 < 4; ++g4)
                *(float4 *)(Fc + 8 * g4) =
                    make_float4(cc[4 * g4], cc[4 * g4 + 1], cc[4 * g4 + 2], cc[4 * g4 + 3]);
        }
        __syncthreads();
        // taps of the rays whose positions fall in this chunk
#pragma unroll
        for (int j = 0; j < AS; ++j) {
            const int q = q0[j];
            const bool t0 = q >= c0 && q < c0 + PCH;
            const bool t1 = q + 1 >= c0 && q + 1 < c0 + PCH;
            if (!(t0 || t1)) continue;
            const float a0 = t0 ? w0[j] : 0.f, a1 = t1 ? w1[j] : 0.f;
            const float *Fj = fr + (j * Npi) * cstride + SF_PAD + (q - c0);   // slot of q
#pragma unroll
            for (int r = 0; r < NPM; ++r) {
                if (r < Npi) {
                    const float x0 = Fj[r * cstride], x1 = Fj[r * cstride + 1];
                    acc[j][r] = fmaf(a1, x1, fmaf(a0, x0, acc[j][r]));
                }
            }
        }
    }

    // ---- epilogue: every half-turn r of class a lands on bin b (even r) or Ns-1-b (odd r)
    double d2 = 0.0;
    const float inv1s = 1.f / (1.f + E.sigma);
#pragma unroll
    for (int j = 0; j < AS; ++j) {
        const int a = j < A ? gcls[grp * A + j] : -1;
        if (a < 0 || tid >= BT || b >= Ns) continue;
#pragma unroll
        for (int r = 0; r < NPM; ++r) {
            if (r >= Npi) continue;
            const int i = r * E.n0 + a;
            const int bo = (r & 1) ? Ns - 1 - b : b;
            const size_t o = ((size_t)i * Nz + z) * Ns + bo;
            const float v = acc[j][r];
            if (!E.prox) {
                E.out[o] = v;
            } else {
                const float d = v - E.gdata[o];
                d2 += (double)d * (double)d;
                E.out[o] = (E.out[o] + E.sigma * d) * inv1s;
            }
        }
    }
    if (E.part) {
        const double sum = block_sum(d2, sh);
        if (tid == 0) E.part[blockIdx.x] = sum;
    }
}

// Fold-sum on MFMA (v_mfma_f32_16x16x16 bf16): per (class a, slice z) the
// product [Ns bins x Npi half-turns] x [Npi x K], half-turns padded to a
// multiple of 16.  One wave per 16-bin x 16-channel tile.
// A: lane holds bins row = lane%16, half-turns 4*(lane/16) + 0..3 of the
// current 16-chunk; B: Phi rows of those half-turns, channel lane%16;
// C: bins 4*(lane/16) + 0..3, channel lane%16.
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
            v4s av, bh, bl;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + 4 * (lane >> 4) + q;
                float gv = 0.f, pv = 0.f;
                if (r < Npi) {
                    const int i = r * n0 + a;
                    if (bin < Ns) gv = g[((size_t)i * Nz + z) * Ns + ((r & 1) ? Ns - 1 - bin : bin)];
                    if (kcol < K) pv = phi[(size_t)i * K + kcol];
                }
                av[q] = (short)bf16_rne(gv);
                const unsigned short h = bf16_rne(pv);
                bh[q] = (short)h;
                bl[q] = (short)bf16_rne(pv - bf16_val(h));
            }
            cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bh, cacc, 0, 0, 0);
            cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bl, cacc, 0, 0, 0);
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

template <int NPM, int KB, int AS>
static int launch_sf_t(const Plan &p, const float *f, const SfEpi &E, hipStream_t s, unsigned nb)
{
    const rt_geom &G = p.g;
    const SfCfg &C = p.sf;
    auto kern = k_project_sf<NPM, KB, AS>;
    if (C.lds > 64 * 1024)
        RT_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)C.lds));
    KTimer kt("k_project_sf", s);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(ST), C.lds, s, f, p.d_phi, p.d_gcls_sf, p.d_gwalk_sf,
                       p.d_ccos, p.d_csin, G.N, G.Nz, G.Ns, G.K, C.A, C.ngroups, C.BT, C.nbt,
                       C.PCH, C.cstride, nb, E);
    kt.stop();
    return RT_OK;
}

template <int NPM, int KB>
static int launch_sf_a(const Plan &p, const float *f, const SfEpi &E, hipStream_t s, unsigned nb)
{
    switch (p.sf.A) {
    case 1: return launch_sf_t<NPM, KB, 1>(p, f, E, s, nb);
    case 2: return launch_sf_t<NPM, KB, 2>(p, f, E, s, nb);
    case 3: return launch_sf_t<NPM, KB, 3>(p, f, E, s, nb);
    default: return launch_sf_t<NPM, KB, 4>(p, f, E, s, nb);
    }
}

template <int NPM>
static int launch_sf_k(const Plan &p, const float *f, const SfEpi &E, hipStream_t s, unsigned nb)
{
    switch ((p.g.K + 7) / 8) {
    case 1: return launch_sf_a<NPM, 1>(p, f, E, s, nb);
    case 2: return launch_sf_a<NPM, 2>(p, f, E, s, nb);
    case 3:
    case 4: return launch_sf_a<NPM, 4>(p, f, E, s, nb);
    default: return launch_sf_a<NPM, 8>(p, f, E, s, nb);
    }
}

}  // namespace

unsigned sf_blocks(const Plan &p) { return (unsigned)p.g.Nz * p.sf.ngroups * p.sf.nbt; }

int launch_forward_sf(const Plan &p, const float *f, float *g, int mode, const float *gdata,
                      float *h1, float sigma, double *part, hipStream_t s)
{
    const rt_geom &G = p.g;
    if (G.Nz == 0) return RT_OK;
    SfEpi E{};
    E.out = mode == CONTRACT_STORE ? g : h1;
    E.gdata = gdata;
    E.part = part;
    E.sigma = sigma;
    E.prox = mode == CONTRACT_PROX;
    E.n0 = p.n0;
    E.Npi = G.Npi;
    const unsigned nb = sf_blocks(p);
    int rc;
    const int npm = p.sf.NPM;
    if (npm <= 4) rc = launch_sf_k<4>(p, f, E, s, nb);
    else if (npm <= 8) rc = launch_sf_k<8>(p, f, E, s, nb);
    else if (npm <= 12) rc = launch_sf_k<12>(p, f, E, s, nb);
    else if (npm <= 16) rc = launch_sf_k<16>(p, f, E, s, nb);
    else rc = launch_sf_k<32>(p, f, E, s, nb);
    if (rc) return rc;
    RT_HIP(hipGetLastError());
    return RT_OK;
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
