// HIP kernels for gfx950 (MI355X) of the fused subdomain training step of
// domain-decomposed PINN flow reconstruction (arXiv 2602.15883).
//
// Method (section 2.1, 2.2): a tanh MLP local expert (x, t) -> (u, p); the
// Navier-Stokes residuals r1..r4 need d/dx_j, d/dt and d2/dx_j^2 of every
// output, which the forward pass carries as extra "channels" through every
// layer (chain rule of tanh); losses L_obs, L_PDE, L_gh_u, L_gh_p (space and
// time parts) and the optional anchor term; hand-written adjoint; Adam
// (Algorithm 1, optimizer step).
//
// Work decomposition
//   A tile holds NCB column blocks of 16 columns.  A collocation tile has
//   16*PBP points and one column block per (channel, 16 points); a value tile
//   (observation, ghost or anchor points, value channel only) has 16*NCB
//   points.  A workgroup of min(Wp/16, 8) waves processes one tile at a
//   time; wave w owns the row block of neurons [16w, 16w+16) of every layer
//   and, for widths above 128 (more than 8 row blocks), also row block w+8.
//   The register footprint per wave stays that of one row block: the wave
//   runs its two blocks one after the other.
//
//   Each hidden layer is Z = W_l H (all channels at once, N = 16*NCB columns)
//   on FP32 MFMA 16x16x4.  The A operand (weights) streams from a
//   fragment-ordered copy in global memory (L2 resident); the B operand
//   (activations) is staged in LDS.  The tanh chain rule runs in registers on
//   the accumulator fragment: lane (g, j) holds rows 16w+4g+i (i = 0..3) of
//   column 16cb+j, so every channel of a (neuron, point) pair sits in one lane.
//
//   Backward: pre-activations z of every layer are stashed per tile in a
//   per-workgroup global ring; the adjoint recomputes tanh and its
//   derivatives from them.  dW_l = Zbar H_{l-1}^T (K = columns) and
//   Hbar_{l-1} = W_l^T Zbar run on MFMA.  Each workgroup accumulates its
//   gradient contribution in a private slab (one per (workgroup, subdomain)
//   segment); a second kernel sums the slabs in a fixed order and applies
//   Adam.  No float atomics: every slab float has one writer lane and the sum
//   order is fixed, so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ddpinn_internal.h"

namespace ddp {

typedef float v4f __attribute__((ext_vector_type(4)));

enum : int { M_PDE = 0, M_VALUE = 1, M_GRAD = 2 };

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4f zero4() { return v4f{0.f, 0.f, 0.f, 0.f}; }

// Accesses to device memory through the global address space: generic
// (flat) accesses would also count against the LDS wait counter, so every
// LDS wait would also wait for outstanding memory loads.
#define GLOBAL_AS __attribute__((address_space(1)))
// read-only for the whole launch (work items, subdomain descriptors): loads
// through the constant address space become scalar loads
#define CONST_AS __attribute__((address_space(4)))
__device__ __forceinline__ v4f ldg4(const float* p) { return *(const GLOBAL_AS v4f*)p; }
__device__ __forceinline__ float ldg(const float* p) { return *(const GLOBAL_AS float*)p; }
__device__ __forceinline__ void stg4(float* p, v4f v) { *(GLOBAL_AS v4f*)p = v; }
__device__ __forceinline__ void stg(float* p, float v) { *(GLOBAL_AS float*)p = v; }
// wave-uniform base + 32-bit per-lane byte offset: selects the scalar-base
// addressing form (one lane-offset register instead of a 64-bit address per lane)
__device__ __forceinline__ v4f ldg4u(const float* base, uint32_t off) {
  return *(const GLOBAL_AS v4f*)((const GLOBAL_AS char*)base + off);
}
__device__ __forceinline__ void stg4u(float* base, uint32_t off, v4f v) {
  *(GLOBAL_AS v4f*)((GLOBAL_AS char*)base + off) = v;
}

// sin and cos with full range reduction (device library)
__device__ __forceinline__ void sincos_f32(float z, float& s, float& c) { sincosf(z, &s, &c); }

// tanh without branches, from two textbook forms:
//   |x| < 0.4 : x * P(x^2), P = Maclaurin series of tanh(x)/x through the x^12
//               term (the first omitted term is below 4e-9 relative)
//   otherwise : sign(x) * (1 - 2 / (exp(2|x|) + 1)), hardware exp2 and rcp
// Within ~3 ulp of the exact value over the whole float range (the float32
// error of this scheme is pinned on the CPU).
__device__ __forceinline__ float tanh_f32(float x) {
  const float a = fabsf(x);
  const float u = x * x;
  float p = 3.5921280365724810e-3f;          //  21844/6081075
  p = fmaf(p, u, -8.8632355299021966e-3f);   // -1382/155925
  p = fmaf(p, u, 2.1869488536155203e-2f);    //  62/2835
  p = fmaf(p, u, -5.3968253968253968e-2f);   // -17/315
  p = fmaf(p, u, 1.3333333333333333e-1f);    //  2/15
  p = fmaf(p, u, -3.3333333333333333e-1f);   // -1/3
  p = fmaf(p, u, 1.f);
  const float small = x * p;
  const float e = __builtin_amdgcn_exp2f(a * 2.8853900817779268f);   // exp(2|x|)
  const float big = __builtin_copysignf(fmaf(-2.f, __builtin_amdgcn_rcpf(e + 1.f), 1.f), x);
  return a < 0.4f ? small : big;
}

enum : int { ACT_TANH = 0, ACT_SIN = 1 };

// activation sigma(z) and its first derivatives: tanh (section 2.1 networks)
// or sin (the paper's cylinder networks, section 3.2-3.3)
template <int ACT>
__device__ __forceinline__ void act_d2(float z, float& s, float& s1, float& s2) {
  if constexpr (ACT == ACT_SIN) {
    sincos_f32(z, s, s1);
    s2 = -s;
  } else {
    s = tanh_f32(z);
    s1 = 1.f - s * s;
    s2 = -2.f * s * s1;
  }
}

// SV: the argument is tanh(z0) itself (kept in the stash in place of z0);
// tanh's derivatives are polynomials in it, so tanh is not evaluated again
template <int ACT, bool SV>
__device__ __forceinline__ void act_d2s(float v, float& s, float& s1, float& s2) {
  if constexpr (SV && ACT == ACT_TANH) {
    s = v;
    s1 = 1.f - s * s;
    s2 = -2.f * s * s1;
  } else {
    act_d2<ACT>(v, s, s1, s2);
  }
}

template <int ACT>
__device__ __forceinline__ void act_d3(float z, float& s, float& s1, float& s2, float& s3) {
  if constexpr (ACT == ACT_SIN) {
    sincos_f32(z, s, s1);
    s2 = -s;
    s3 = -s1;
  } else {
    s = tanh_f32(z);
    s1 = 1.f - s * s;
    s2 = -2.f * s * s1;
    s3 = 2.f * s1 * (3.f * s * s - 1.f);
  }
}

template <int ACT, bool SV>
__device__ __forceinline__ void act_d3s(float v, float& s, float& s1, float& s2, float& s3) {
  if constexpr (SV && ACT == ACT_TANH) {
    s = v;
    s1 = 1.f - s * s;
    s2 = -2.f * s * s1;
    s3 = 2.f * s1 * (3.f * s * s - 1.f);
  } else {
    act_d3<ACT>(v, s, s1, s2, s3);
  }
}

// Channel layout of a tile in a given mode.
//   M_PDE  : CM = 2d+2 channels: 0 value, 1..d d/dx_j, d+1 d/dt, d+2..2d+1 d2/dx_j^2
//   M_GRAD : CM = d+1 channels: 0 value, 1..d d/dx_j
//   M_VALUE: CM = 1
// Column block of (channel c, point block pb) = c*NPB + pb.
template <int DIM, int NCB, int MODE>
struct ModeCfg {
  static constexpr int CF = 2 * DIM + 2;
  static constexpr int CM = MODE == M_PDE ? CF : (MODE == M_VALUE ? 1 : DIM + 1);
  static constexpr int NPB = NCB / CM;
  static constexpr int NPTS = 16 * NPB;
  static_assert(NCB % CM == 0, "column blocks must hold whole channel sets");
};

// ---------------------------------------------------------------------------
// activation: z -> h with the chain rule, in place on accumulator fragments
//   h = sigma(z0); h_j = s1 z_j; h_jj = s2 z_j^2 + s1 z_jj
//   s1, s2 = first and second derivative of sigma at z0
// ---------------------------------------------------------------------------
template <int DIM, int NCB, int MODE, int ACT>
__device__ __forceinline__ void act_forward(v4f (&a)[NCB]) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int NPB = M::NPB;
#pragma unroll
  for (int pb = 0; pb < NPB; ++pb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float s, s1, s2;
      act_d2<ACT>(a[pb][i], s, s1, s2);
      if constexpr (MODE == M_PDE) {
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) {
          const float z1 = a[(1 + jj) * NPB + pb][i];
          const float z2 = a[(DIM + 2 + jj) * NPB + pb][i];
          a[(DIM + 2 + jj) * NPB + pb][i] = s2 * z1 * z1 + s1 * z2;
        }
#pragma unroll
        for (int jj = 0; jj <= DIM; ++jj) a[(1 + jj) * NPB + pb][i] *= s1;
      } else if constexpr (MODE == M_GRAD) {
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) a[(1 + jj) * NPB + pb][i] *= s1;
      }
      a[pb][i] = s;
    }
  }
}

// h = act(z) of a stashed pre-activation stack, written straight into the
// neuron-major LDS layout [neuron][column] (stride S2) used by the dW GEMM.
template <int DIM, int NCB, int MODE, int ACT>
__device__ __forceinline__ void act_store_bwd(float* buf, int S2, const v4f (&z)[NCB], int w, int g, int j) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int NPB = M::NPB;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float* row = buf + (16 * w + 4 * g + i) * S2 + j;
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb) {
      float s, s1, s2;
      act_d2<ACT>(z[pb][i], s, s1, s2);
      row[16 * pb] = s;
      if constexpr (MODE == M_PDE) {
#pragma unroll
        for (int jj = 0; jj <= DIM; ++jj) row[16 * ((1 + jj) * NPB + pb)] = s1 * z[(1 + jj) * NPB + pb][i];
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) {
          const float z1 = z[(1 + jj) * NPB + pb][i];
          row[16 * ((DIM + 2 + jj) * NPB + pb)] = s2 * z1 * z1 + s1 * z[(DIM + 2 + jj) * NPB + pb][i];
        }
      }
    }
  }
}

// Adjoint of act_forward: hb (dL/dh) -> dL/dz in place; zs holds z.
//   zbar_jj = s1 hbar_jj
//   zbar_j  = s1 hbar_j + 2 s2 z_j hbar_jj      (spatial j; time: s1 hbar_t)
//   zbar_0  = s1 hbar_0 + s2 sum_j z_j hbar_j + sum_j (s3 z_j^2 + s2 z_jj) hbar_jj
//   with s1, s2, s3 the first three derivatives of the activation at z_0
template <int DIM, int NCB, int MODE, int ACT, bool SV = false>
__device__ __forceinline__ void act_adjoint(v4f (&hb)[NCB], const v4f (&zs)[NCB]) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int NPB = M::NPB;
#pragma unroll
  for (int pb = 0; pb < NPB; ++pb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if constexpr (MODE == M_PDE) {
        float s, s1, s2, s3;
        act_d3s<ACT, SV>(zs[pb][i], s, s1, s2, s3);
        float z0b = s1 * hb[pb][i];
#pragma unroll
        for (int jj = 0; jj <= DIM; ++jj) {
          const int c = (1 + jj) * NPB + pb;
          const float h1 = hb[c][i];
          z0b += s2 * zs[c][i] * h1;
          hb[c][i] = s1 * h1;
        }
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) {
          const int c1 = (1 + jj) * NPB + pb, c2 = (DIM + 2 + jj) * NPB + pb;
          const float h2 = hb[c2][i];
          const float z1 = zs[c1][i], z2 = zs[c2][i];
          hb[c2][i] = s1 * h2;
          hb[c1][i] += 2.f * s2 * z1 * h2;
          z0b += (s3 * z1 * z1 + s2 * z2) * h2;
        }
        hb[pb][i] = z0b;
      } else {
        float s, s1, s2;
        act_d2s<ACT, SV>(zs[pb][i], s, s1, s2);
        hb[pb][i] *= s1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// GEMMs on FP32 MFMA 16x16x4
//
// K index of MFMA step s in lane group g (g = lane/16): kmap(s, g) = g*Wq + s
// with Wq = Wp/4, so that 4 consecutive steps of one lane read 4 contiguous
// floats (one ds_read_b128).  The weight fragments are laid out with the same
// map:  frag[((w*K4 + s4)*64 + lane)*4 + q] = W[16w + lane%16][kmap(4 s4 + q, lane/16)].
// ---------------------------------------------------------------------------

// acc[cb] += A(16 rows of this wave) * B(LDS [16*NCB cols][S], K = Wp).
// With TR the same operands enter the MFMA the other way round: the LDS
// activations are the A operand and the weight fragment the B operand, so
// acc[cb] holds the transposed tile (lane (g, j): column 16cb + 4g + i,
// neuron 16w + j) from the same loads.
template <bool TR>
__device__ __forceinline__ v4f mfma_or(const float wf, const float act, v4f c) {
  return TR ? mfma4(act, wf, c) : mfma4(wf, act, c);
}

template <int NCB, bool TR = false>
__device__ __forceinline__ void mfma_step(const v4f a, const float* bb, int S, int s4, v4f (&acc)[NCB]) {
  v4f b[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) b[cb] = *reinterpret_cast<const v4f*>(bb + cb * 16 * S + 4 * s4);
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma_or<TR>(a[q], b[cb][q], acc[cb]);
}

// the last, partial chunk: only its first KT K-steps hold neurons
template <int NCB, bool TR = false>
__device__ __forceinline__ void mfma_tail(const v4f a, const float* bb, int S, int s4, int KT, v4f (&acc)[NCB]) {
  v4f b[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) b[cb] = *reinterpret_cast<const v4f*>(bb + cb * 16 * S + 4 * s4);
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma_or<TR>(a[0], b[cb][0], acc[cb]);
  if (KT > 1) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma_or<TR>(a[1], b[cb][1], acc[cb]);
  }
  if (KT > 2) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma_or<TR>(a[2], b[cb][2], acc[cb]);
  }
}

// K = 4*K4 + KT steps: K4 full chunks of four, then KT (0..3) more
// INIT: acc is written, not accumulated into: the first MFMA of each
// accumulator takes 0 as its C operand (no zeroing of the accumulators)
template <int NCB, bool TR = false, bool INIT = false, bool DEEP = false>
__device__ __forceinline__ void gemm_rows(const float* __restrict__ afrag, const float* bufB,
                                          int S, int K4, int g, int j, int lane,
                                          v4f (&acc)[NCB], int KT) {
  const int KC = K4 + (KT ? 1 : 0);   // chunks per row block (4*KC = Wp/4, a lane group's segment)
  const float* bb = bufB + j * S + g * (4 * KC);
  const uint32_t lo = (uint32_t)lane * 16u;
  // DEEP: three weight-fragment registers, the fragments of the next two
  // chunks are in flight while the MFMAs of the current one run (one chunk's
  // MFMAs do not always cover the latency of a fragment read from L2);
  // otherwise two (for kernels without the four registers to spare).
  // Chunks past the last re-read the last one.
  auto frag = [&](int c) { return ldg4u(afrag + (c < KC ? c : KC - 1) * 256, lo); };
  v4f a0 = frag(0);
  v4f a1 = frag(1);
  int s4 = 0;
  if constexpr (INIT) {
    v4f b[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) b[cb] = *reinterpret_cast<const v4f*>(bb + cb * 16 * S);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma_or<TR>(a0[0], b[cb][0], zero4());
    const int q1 = K4 > 0 ? 4 : KT;   // K-steps of the first chunk
    if (q1 > 1) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma_or<TR>(a0[1], b[cb][1], acc[cb]);
    }
    if (q1 > 2) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma_or<TR>(a0[2], b[cb][2], acc[cb]);
    }
    if (q1 > 3) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma_or<TR>(a0[3], b[cb][3], acc[cb]);
    }
    if (K4 == 0) return;
    s4 = 1;
    a0 = a1;
    a1 = frag(2);
  }
  if constexpr (!DEEP) {
    // a0, a1: the fragments of chunks s4 and s4 + 1
    for (; s4 + 2 <= K4; s4 += 2) {
      mfma_step<NCB, TR>(a0, bb, S, s4, acc);
      a0 = frag(s4 + 2);
      mfma_step<NCB, TR>(a1, bb, S, s4 + 1, acc);
      a1 = frag(s4 + 3);
    }
    if (s4 < K4) {
      mfma_step<NCB, TR>(a0, bb, S, s4, acc);
      a0 = a1;
      ++s4;
    }
    if (KT) mfma_tail<NCB, TR>(a0, bb, S, s4, KT, acc);
    return;
  }
  // a0, a1: the fragments of chunks s4 and s4 + 1
  for (; s4 + 3 <= K4; s4 += 3) {
    const v4f a2 = frag(s4 + 2);
    mfma_step<NCB, TR>(a0, bb, S, s4, acc);
    a0 = frag(s4 + 3);
    mfma_step<NCB, TR>(a1, bb, S, s4 + 1, acc);
    a1 = frag(s4 + 4);
    mfma_step<NCB, TR>(a2, bb, S, s4 + 2, acc);
  }
  if (s4 < K4) {
    const v4f a2 = frag(s4 + 2);
    mfma_step<NCB, TR>(a0, bb, S, s4, acc);
    a0 = a1;
    a1 = a2;
    ++s4;
  }
  if (s4 < K4) {
    mfma_step<NCB, TR>(a0, bb, S, s4, acc);
    a0 = a1;
    ++s4;
  }
  if (KT) mfma_tail<NCB, TR>(a0, bb, S, s4, KT, acc);
}

// acc = the rows of one row block over the K chunks [c0, c1) of the KC
// chunks of a lane group's segment (the last chunk holds KT steps if KT > 0):
// one part of a GEMM whose K range is split between waves
template <int NCB>
__device__ __forceinline__ void gemm_rows_part(const float* __restrict__ afrag, const float* bufB, int S, int KC,
                                               int KT, int c0, int c1, int g, int j, int lane, v4f (&acc)[NCB]) {
  const float* bb = bufB + j * S + g * (4 * KC);
  const uint32_t lo = (uint32_t)lane * 16u;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = zero4();
  v4f a = ldg4u(afrag + c0 * 256, lo);
  for (int c = c0; c < c1; ++c) {
    const v4f an = (c + 1 < c1) ? ldg4u(afrag + (c + 1) * 256, lo) : a;
    if (c == KC - 1 && KT) mfma_tail<NCB>(a, bb, S, c, KT, acc);
    else mfma_step<NCB>(a, bb, S, c, acc);
    a = an;
  }
}

// dw[t] += sum_col Zbar[16w + m][col] * Hprev[16(nb0+t) + n][col], t < NNB
//   Zbar from bufG ([col][neuron], stride S); Hprev from bufHb ([neuron][col], stride S2)
//   Column of step (s4, q) in lane group g: 16*s4 + 4*g + q.  The four groups
//   then read Zbar rows 4*S apart (S = Wp + 4 = 4 mod 16, so 16 banks apart):
//   the 64 lanes of one A read hit 64 distinct banks; a group's B read is 4
//   contiguous columns of a neuron row (one ds_read_b128).
template <int NCB, int NNB>
__device__ __forceinline__ void gemm_dw(const float* bufG, int S, const float* bufHb, int S2,
                                        int w, int g, int j, int nb0, v4f (&dw)[4]) {
  const float* ab = bufG + (4 * g) * S + 16 * w + j;
  const float* bb = bufHb + (16 * nb0 + j) * S2 + 4 * g;
  for (int s4 = 0; s4 < NCB; ++s4) {
    float a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = ab[(16 * s4 + q) * S];
    v4f b[NNB];
#pragma unroll
    for (int t = 0; t < NNB; ++t) b[t] = *reinterpret_cast<const v4f*>(bb + t * 16 * S2 + 16 * s4);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < NNB; ++t) dw[t] = mfma4(a[q], b[t][q], dw[t]);
  }
}

// sum over the 16 lanes of a lane group (same g)
__device__ __forceinline__ float sum16(float v) {
  v += __shfl_xor(v, 8, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 1, 16);
  return v;
}

// sum over the four lane groups (same j)
__device__ __forceinline__ float sum_groups(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Transposed tiles (the one-row-block step kernel).  Every GEMM of that kernel
// enters its operands the other way round (gemm_rows<NCB, true>), so a wave's
// accumulator fragment acc[cb] holds, in lane (g, j), neuron 16w + j of
// columns 16cb + 4g + i (i = 0..3).  Every channel of a (neuron, point) pair
// still sits in one lane (column block cb = channel), so the chain rule runs
// in registers as before, and the weight gradient
//   dW_l[16w + m][n] = sum_col Zbar_l[16w + m][col] H_{l-1}[n][col]
// takes its A operand (Zbar_l of this wave's neurons, K = columns) straight
// from the registers: step (cb, i) pairs lane (g, j)'s acc[cb][i] with
// column 16cb + 4g + i.  Only H_{l-1} comes from LDS, four columns per
// ds_read_b128.
// ---------------------------------------------------------------------------

// input layer: z0 = W1 xi + b1 and the seeded channels, transposed tile
template <int DIM, int NCB, int MODE>
__device__ __forceinline__ void input_layer_t(v4f (&a)[NCB], const float* __restrict__ W1p,
                                              const float* __restrict__ b1p, const float* xin,
                                              int w, int g, int j) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int D = DIM + 1, NPB = M::NPB;
  const int r = 16 * w + j;
  float wr[D];
#pragma unroll
  for (int q = 0; q < D; ++q) wr[q] = ldg(W1p + r * D + q);
  const float br = ldg(b1p + r);
#pragma unroll
  for (int pb = 0; pb < NPB; ++pb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float* xp = xin + (16 * pb + 4 * g + i) * D;
      float z = br;
#pragma unroll
      for (int q = 0; q < D; ++q) z += wr[q] * xp[q];
      a[pb][i] = z;
    }
    if constexpr (MODE == M_PDE) {
#pragma unroll
      for (int jj = 0; jj <= DIM; ++jj) a[(1 + jj) * NPB + pb] = v4f{wr[jj], wr[jj], wr[jj], wr[jj]};
#pragma unroll
      for (int jj = 0; jj < DIM; ++jj) a[(DIM + 2 + jj) * NPB + pb] = zero4();
    } else if constexpr (MODE == M_GRAD) {
#pragma unroll
      for (int jj = 0; jj < DIM; ++jj) a[(1 + jj) * NPB + pb] = v4f{wr[jj], wr[jj], wr[jj], wr[jj]};
    }
  }
}

// add the bias of this lane's neuron to the value-channel column blocks
template <int NCB, int NPB>
__device__ __forceinline__ void add_bias_t(v4f (&a)[NCB], const float* __restrict__ b, int w, int j) {
  const float bv = ldg(b + 16 * w + j);
#pragma unroll
  for (int pb = 0; pb < NPB; ++pb) a[pb] += bv;
}

// store a transposed fragment into the LDS layout [col][neuron] (stride S)
template <int NCB>
__device__ __forceinline__ void store_fwd_t(float* buf, int S, const v4f (&a)[NCB], int w, int g, int j) {
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int i = 0; i < 4; ++i) buf[(16 * cb + 4 * g + i) * S + 16 * w + j] = a[cb][i];
}

// h = act(z) of a stashed (transposed) pre-activation stack, written into the
// neuron-major LDS layout [neuron][col] (stride S2): four columns per store
template <int DIM, int NCB, int MODE, int ACT, bool SV = false>
__device__ __forceinline__ void act_store_bwd_t(float* buf, int S2, const v4f (&z)[NCB], int w, int g, int j) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int NPB = M::NPB;
  float* row = buf + (16 * w + j) * S2 + 4 * g;
#pragma unroll
  for (int pb = 0; pb < NPB; ++pb) {
    // activation derivatives of the four columns first, then one channel
    // at a time into a four-column store (few values live at once)
    v4f sv, s1, s2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float a0, a1, a2;
      act_d2s<ACT, SV>(z[pb][i], a0, a1, a2);
      sv[i] = a0;
      s1[i] = a1;
      s2[i] = a2;
    }
    *reinterpret_cast<v4f*>(row + 16 * pb) = sv;
    if constexpr (MODE == M_PDE) {
#pragma unroll
      for (int jj = 0; jj <= DIM; ++jj)
        *reinterpret_cast<v4f*>(row + 16 * ((1 + jj) * NPB + pb)) = s1 * z[(1 + jj) * NPB + pb];
#pragma unroll
      for (int jj = 0; jj < DIM; ++jj) {
        const v4f z1 = z[(1 + jj) * NPB + pb];
        *reinterpret_cast<v4f*>(row + 16 * ((DIM + 2 + jj) * NPB + pb)) = s2 * z1 * z1 + s1 * z[(DIM + 2 + jj) * NPB + pb];
      }
    }
  }
}

// dw[t] = Zbar(this wave's neurons, registers) * Hprev[16(nb0+t) + n][.]^T,
// t < NNB (the first MFMA takes 0 as its C operand)
//   Hprev from bufHb ([neuron][col], stride S2); K = the tile's columns
template <int NCB, int NNB>
__device__ __forceinline__ void gemm_dw_t(const v4f (&zb)[NCB], const float* bufHb, int S2, int g, int j,
                                          int nb0, v4f (&dw)[4]) {
  const float* bb = bufHb + (16 * nb0 + j) * S2 + 4 * g;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    v4f b[NNB];
#pragma unroll
    for (int t = 0; t < NNB; ++t) b[t] = *reinterpret_cast<const v4f*>(bb + t * 16 * S2 + 16 * cb);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int t = 0; t < NNB; ++t) dw[t] = mfma4(zb[cb][i], b[t][i], (cb == 0 && i == 0) ? zero4() : dw[t]);
  }
}

// ---------------------------------------------------------------------------
// shared forward pieces
// ---------------------------------------------------------------------------

// input layer: z0 = W1 xi + b1; z_j = W1[:, j] (first-derivative channels);
// second-derivative channels start at 0.  xin: LDS [points][D].
template <int DIM, int NCB, int MODE>
__device__ __forceinline__ void input_layer(v4f (&a)[NCB], const float* __restrict__ W1p,
                                            const float* __restrict__ b1p, const float* xin,
                                            int w, int g, int j) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int D = DIM + 1, NPB = M::NPB;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * w + 4 * g + i;
    float wr[D];
#pragma unroll
    for (int q = 0; q < D; ++q) wr[q] = ldg(W1p + r * D + q);
    const float br = ldg(b1p + r);
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb) {
      const float* xp = xin + (16 * pb + j) * D;
      float z = br;
#pragma unroll
      for (int q = 0; q < D; ++q) z += wr[q] * xp[q];
      a[pb][i] = z;
      if constexpr (MODE == M_PDE) {
#pragma unroll
        for (int jj = 0; jj <= DIM; ++jj) a[(1 + jj) * NPB + pb][i] = wr[jj];
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) a[(DIM + 2 + jj) * NPB + pb][i] = 0.f;
      } else if constexpr (MODE == M_GRAD) {
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) a[(1 + jj) * NPB + pb][i] = wr[jj];
      }
    }
  }
}

// store an accumulator fragment into the forward LDS layout [col][neuron]
template <int NCB>
__device__ __forceinline__ void store_fwd(float* buf, int S, const v4f (&a)[NCB], int w, int g, int j) {
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
    *reinterpret_cast<v4f*>(buf + (16 * cb + j) * S + 16 * w + 4 * g) = a[cb];
}

// add the bias to the value-channel column blocks
template <int NCB, int NPB>
__device__ __forceinline__ void add_bias(v4f (&a)[NCB], const float* __restrict__ b, int w, int g) {
  const v4f bv = ldg4(b + 16 * w + 4 * g);
#pragma unroll
  for (int pb = 0; pb < NPB; ++pb) a[pb] += bv;
}

// output layer: ys[o][col] = W_{H+1}[o] . h[col] (+ b_{H+1}[o] on value columns)
template <int DIM, int NCB, int MODE>
__device__ __forceinline__ void output_layer(const float* bufH, int S, int Wp,
                                             const float* __restrict__ Wop, const float* __restrict__ bop,
                                             float* ys, int tid, int nthr) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int D = DIM + 1, NCOL = 16 * NCB;
  for (int idx = tid; idx < D * NCOL; idx += nthr) {
    const int o = idx / NCOL, col = idx - o * NCOL;
    const float* hr = bufH + col * S;
    const float* wo = Wop + o * Wp;
    float acc = 0.f;
    for (int n = 0; n < Wp; n += 4) {
      const v4f h4 = *reinterpret_cast<const v4f*>(hr + n);
      const v4f w4 = ldg4(wo + n);
      acc += h4[0] * w4[0];
      acc += h4[1] * w4[1];
      acc += h4[2] * w4[2];
      acc += h4[3] * w4[3];
    }
    if (col < 16 * M::NPB) acc += ldg(bop + o);
    ys[o * NCOL + col] = acc;
  }
}

// Navier-Stokes residuals r1..r_{d+1} (section 2.1) from the channel stack of
// one point; Y(c, o) = output o of channel c.
template <int DIM, typename F>
__device__ __forceinline__ void residuals(F Y, float nu, float (&r)[DIM + 1]) {
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    float conv = 0.f, lap = 0.f;
#pragma unroll
    for (int jj = 0; jj < DIM; ++jj) {
      conv += Y(0, jj) * Y(1 + jj, i);
      lap += Y(DIM + 2 + jj, i);
    }
    r[i] = Y(1 + DIM, i) + conv + Y(1 + i, DIM) - nu * lap;
  }
  float div = 0.f;
#pragma unroll
  for (int jj = 0; jj < DIM; ++jj) div += Y(1 + jj, jj);
  r[DIM] = div;
}

// ---------------------------------------------------------------------------
// LDS plan of the step kernel (floats)
// ---------------------------------------------------------------------------
struct StepLds {
  int S, S2, NCOL;
  int bufH, bufG, ys, yb, xin, acc1, dbacc, red, sched, part, nparts, total;
};

// Row blocks beyond the eight waves.  With exactly two of them (Wp = 160, the
// paper's 6x150 network) the plan with two stacks per tile splits their
// GEMMs' K range in halves between four waves, one per SIMD, so no wave
// carries more than 1.5 row blocks (instead of 2, 2, 1, ...) and every SIMD
// 2.5 (instead of 3, 3, 2, 2).  The parts meet in four LDS tiles; only where
// those fit in the 160 KB of LDS as well.
constexpr int kLdsBytes = 160 * 1024;
__host__ __device__ inline int step_ksplit_parts(int Wp, int split, int floats_before, int NCB) {
  const int nw = Wp / 16, ne = nw - (nw < 8 ? nw : 8);
  const bool want = !split && ne == 2;
  return (want && (floats_before + 4 * NCB * 256) * 4 <= kLdsBytes) ? 4 : 0;
}

// Row stride of the [col][neuron] stacks.  Up to 128 neurons it is a
// compile-time constant per kernel instance (68, 100 or 132 floats, the
// smallest that holds Wp + 4); above, Wp + 4, a compile-time constant for the
// paper's cylinder widths (Wp = 160 and 208) and a kernel argument for the
// others.  A constant stride makes every LDS address of a tile one lane base
// plus an immediate offset.  With each stride the rows that one operand read
// or store touches fall in distinct banks.
__host__ __device__ inline int step_row_stride(int Wp) {
  return Wp <= 64 ? 68 : (Wp <= 96 ? 100 : (Wp <= 128 ? 132 : Wp + 4));
}

__host__ __device__ inline StepLds step_lds(int D, int Wp, int H, int NCB, int S = 0) {
  StepLds L;
  L.NCOL = 16 * NCB;
  L.S = S ? S : Wp + 4;
  L.S2 = L.NCOL + 4;
  const int hsz = (L.NCOL * L.S > Wp * L.S2) ? L.NCOL * L.S : Wp * L.S2;
  int o = 0;
  L.bufH = o; o += (hsz + 3) & ~3;
  L.bufG = o; o += (L.NCOL * L.S + 3) & ~3;
  L.ys = o;   o += (D * L.NCOL + 3) & ~3;
  L.yb = o;   o += (D * L.NCOL + 3) & ~3;
  L.xin = o;  o += (L.NCOL * D + 3) & ~3;
  L.acc1 = o; o += (Wp * D + 3) & ~3;
  L.dbacc = o; o += (H * Wp + 3) & ~3;
  L.red = o;  o += 64;
  L.sched = o; o += 4;   // the item range taken by the workgroup
  L.part = o;
  L.nparts = step_ksplit_parts(Wp, 0, o, NCB);
  o += L.nparts * NCB * 256;
  L.total = o;
  return L;
}

// LDS plan of the column-split variant (two row blocks per wave, when the
// plan above does not fit): the forward keeps one activation stack [NCOL][S]
// at bufG; the backward holds Zbar [NCOL/2][S] at bufG and H_{l-1}
// [Wp][NCOL/2 + 4] at bufH for one half of the tile's columns at a time.
__host__ __device__ inline StepLds step_lds_split(int D, int Wp, int H, int NCB, int S = 0) {
  StepLds L;
  L.NCOL = 16 * NCB;
  L.S = S ? S : Wp + 4;
  L.S2 = L.NCOL / 2 + 4;
  const int zh = ((L.NCOL / 2) * L.S + 3) & ~3;
  const int bwd = zh + Wp * L.S2;
  const int fwd = L.NCOL * L.S;
  int o = 0;
  L.bufG = o;
  L.bufH = o + zh;
  o += ((fwd > bwd ? fwd : bwd) + 3) & ~3;
  L.ys = o;   o += (D * L.NCOL + 3) & ~3;
  L.yb = o;   o += (D * L.NCOL + 3) & ~3;
  L.xin = o;  o += (L.NCOL * D + 3) & ~3;
  L.acc1 = o; o += (Wp * D + 3) & ~3;
  L.dbacc = o; o += (H * Wp + 3) & ~3;
  L.red = o;  o += 64;
  L.sched = o; o += 4;
  L.part = o;
  L.nparts = step_ksplit_parts(Wp, 1, o, NCB);
  o += L.nparts * NCB * 256;
  L.total = o;
  return L;
}

// ---------------------------------------------------------------------------
// Backward pieces of one row block, for workgroups whose waves own two row
// blocks (the one-row-block path runs the same steps inline)
// ---------------------------------------------------------------------------

// hbar_H = W_{H+1}^T ybar for the rows of row block rb
template <int D, int NCB>
__device__ __forceinline__ void out_adjoint_rows(v4f (&acc)[NCB], const float* __restrict__ Wop, const float* yb,
                                                 int Wp, int rb, int g, int j) {
  constexpr int NCOL = 16 * NCB;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * rb + 4 * g + i;
    float wo[D];
#pragma unroll
    for (int o = 0; o < D; ++o) wo[o] = ldg(Wop + o * Wp + r);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < D; ++o) s += wo[o] * yb[o * NCOL + 16 * cb + j];
      acc[cb][i] = s;
    }
  }
}

// layer l, row block rb: zbar from hbar (acc, in place) and z_l (zs); db_l;
// at l = 1 the input-layer gradient dW1
template <int DIM, int NCB, int MODE, int ACT>
__device__ __forceinline__ void adjoint_rows(v4f (&acc)[NCB], const v4f (&zs)[NCB], float* dbacc, float* acc1,
                                             const float* xin, int Wp, int rb, int l, int g, int j) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int D = DIM + 1;
  act_adjoint<DIM, NCB, MODE, ACT>(acc, zs);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float s = 0.f;
#pragma unroll
    for (int pb = 0; pb < M::NPB; ++pb) s += acc[pb][i];
    s = sum16(s);
    if (j == 0) dbacc[(l - 1) * Wp + 16 * rb + 4 * g + i] += s;
  }
  if (l != 1) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * rb + 4 * g + i;
    float v[D];
#pragma unroll
    for (int q = 0; q < D; ++q) v[q] = 0.f;
#pragma unroll
    for (int pb = 0; pb < M::NPB; ++pb) {
      const float* xp = xin + (16 * pb + j) * D;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        v[q] += acc[pb][i] * xp[q];
        if constexpr (MODE == M_PDE) v[q] += acc[(1 + q) * M::NPB + pb][i];
      }
    }
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const float s = sum16(v[q]);
      if (j == 0) acc1[r * D + q] += s;
    }
  }
}

template <int SPLIT>
__host__ __device__ inline StepLds step_plan(int D, int Wp, int H, int NCB, int S = 0) {
  if constexpr (SPLIT) return step_lds_split(D, Wp, H, NCB, S);
  else return step_lds(D, Wp, H, NCB, S);
}

// h = act(z) of a stashed pre-activation stack, only the column blocks
// [CB0, CB0 + NCBH), written to the neuron-major LDS layout of that half
template <int DIM, int NCB, int MODE, int ACT, int CB0, int NCBH>
__device__ __forceinline__ void act_store_bwd_cols(float* buf, int S2, const v4f (&z)[NCB], int rb, int g, int j) {
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int NPB = M::NPB;
  auto put = [](float* row, int cb, float v) {
    if (cb >= CB0 && cb < CB0 + NCBH) row[16 * (cb - CB0)] = v;
  };
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float* row = buf + (16 * rb + 4 * g + i) * S2 + j;
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb) {
      if constexpr (MODE != M_PDE) {
        if (pb < CB0 || pb >= CB0 + NCBH) continue;
      }
      float s, s1, s2;
      act_d2<ACT>(z[pb][i], s, s1, s2);
      put(row, pb, s);
      if constexpr (MODE == M_PDE) {
#pragma unroll
        for (int jj = 0; jj <= DIM; ++jj) put(row, (1 + jj) * NPB + pb, s1 * z[(1 + jj) * NPB + pb][i]);
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) {
          const float z1 = z[(1 + jj) * NPB + pb][i];
          put(row, (DIM + 2 + jj) * NPB + pb, s2 * z1 * z1 + s1 * z[(DIM + 2 + jj) * NPB + pb][i]);
        }
      }
    }
  }
}

// dW_l += Zbar_l H_{l-1}^T over the (row block, column block) tiles
// [t0, t1) of the layer, row-major, into the layer's block sw of the
// segment's slab.  A tile reads only LDS (the Zbar rows of its row block, the
// H rows of its column block), so any wave can take any tile: the NW*NW tiles
// are cut into equal contiguous runs, one per wave, which balances the SIMDs
// whatever row blocks their waves own (one writer per slab float still).
// Up to four tiles of one row block share the A operand.  The old slab values
// of a group are requested one group ahead (during the previous group's
// GEMM), so two groups' GEMMs cover the read's latency.
template <int NCB>
__device__ __forceinline__ void dw_tiles(float* sw, bool first, const float* bufG, int S, const float* bufH, int S2,
                                         int NW, int t0, int t1, int g, int j, uint32_t lo16) {
  auto group = [&](int t, int& rb, int& nb0) {
    rb = t / NW;
    nb0 = t - rb * NW;
    const int n = NW - nb0 < 4 ? NW - nb0 : 4;
    return n < t1 - t ? n : t1 - t;
  };
  v4f oldn[4];
  if (t0 < t1) {
    int rb, nb0;
    const int nnb = group(t0, rb, nb0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      oldn[q] = (q < nnb && !first) ? ldg4u(sw + (size_t)(rb * NW + nb0 + q) * 256, lo16) : zero4();
  }
  for (int t = t0; t < t1;) {
    int rb, nb0;
    const int nnb = group(t, rb, nb0);
    v4f old[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) old[q] = oldn[q];
    if (t + nnb < t1 && !first) {
      int rb2, nb2;
      const int n2 = group(t + nnb, rb2, nb2);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        oldn[q] = q < n2 ? ldg4u(sw + (size_t)(rb2 * NW + nb2 + q) * 256, lo16) : zero4();
    }
    v4f dw[4] = {zero4(), zero4(), zero4(), zero4()};
    switch (nnb) {
      case 4: gemm_dw<NCB, 4>(bufG, S, bufH, S2, rb, g, j, nb0, dw); break;
      case 3: gemm_dw<NCB, 3>(bufG, S, bufH, S2, rb, g, j, nb0, dw); break;
      case 2: gemm_dw<NCB, 2>(bufG, S, bufH, S2, rb, g, j, nb0, dw); break;
      default: gemm_dw<NCB, 1>(bufG, S, bufH, S2, rb, g, j, nb0, dw); break;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nnb) stg4u(sw + (size_t)(rb * NW + nb0 + q) * 256, lo16, old[q] + dw[q]);
    t += nnb;
  }
}

// ---------------------------------------------------------------------------
// Fused step kernel: persistent over this workgroup's item range.
// ---------------------------------------------------------------------------
// SS: the row stride of the [col][neuron] stacks (step_row_stride)
template <int DIM, int PBP, int ACT, int RPW, int SPLIT, int SS>
__global__ __launch_bounds__(PBP == 1 ? 512 : 256) void step_kernel(const StepArgs args) {
  constexpr int D = DIM + 1;
  constexpr int CF = 2 * DIM + 2;
  constexpr int NCB = CF * PBP;
  constexpr int NCOL = 16 * NCB;
  using MP = ModeCfg<DIM, NCB, M_PDE>;
  using MV = ModeCfg<DIM, NCB, M_VALUE>;
  extern __shared__ float lds[];

  const Shape& sh = args.sh;
  const int Wp = sh.Wp, NW = sh.NW, NWV = sh.NWV, H = sh.H;
  const int K4 = sh.Kq >> 2, KT = sh.Kq & 3;   // K-steps of the hidden GEMMs: 4*K4 + KT
  const int tid = threadIdx.x, nthr = blockDim.x;
  // the wave index is uniform across a wave: keeping it in a scalar register
  // lets every per-wave address (weights, stash, slab) be a scalar base plus
  // the lane offset instead of a 64-bit vector address per use
  const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4, j = lane & 15;
  const StepLds L = step_plan<SPLIT>(D, Wp, H, NCB, SS);
  float* bufH = lds + L.bufH;
  float* bufG = lds + L.bufG;
  float* ys = lds + L.ys;
  float* yb = lds + L.yb;
  float* xin = lds + L.xin;
  float* acc1 = lds + L.acc1;
  float* dbacc = lds + L.dbacc;
  float* red = lds + L.red;
  float* part = lds + L.part;
  const int S = SS ? SS : L.S, S2 = L.S2;
  // two row blocks beyond the eight waves (the plan with two stacks per tile): their GEMMs are
  // split over K between waves w and w + 2 (w < 2, the blocks' owners), and
  // summed by the owner from four LDS tiles
  const bool ks = RPW == 2 && !SPLIT && L.nparts == 4;
  const int KCh = ((sh.Kq + 3) >> 2);   // K chunks of a lane group's segment
  // dW tiles of this wave (two-row-block kernels): the layer's NW*NW tiles in
  // contiguous runs whose lengths even out each wave's work between two
  // barriers.  A row block of Hbar costs NW dW tiles in multiply-adds (both
  // run over the same columns), and its share of the per-row-block VALU work
  // around the GEMMs (recomputing h, the adjoint) adds about a quarter of
  // that; so a wave with fewer Hbar row blocks takes more dW tiles: wave v's
  // share is (9/4 NW^2 - 5/4 NWV * NW * rows(v)) / NWV, rows(v) its row
  // blocks (1.5 for waves 0..3 with the K-split above).  cut(v) is the sum
  // of the shares of waves < v, with rows counted in halves.
  auto dw_cut = [&](int v) {
    const int ne = NW - NWV;
    const int hb = ks ? 3 * (v < 4 ? v : 4) + 2 * (v > 4 ? v - 4 : 0) : 2 * v + 2 * (v < ne ? v : ne);
    return (18 * NW * NW * v - 5 * NW * NWV * hb) / (8 * NWV);
  };
  const int dw_t0 = (RPW == 2) ? dw_cut(w) : 0, dw_t1 = (RPW == 2) ? dw_cut(w + 1) : 0;

  // row blocks of this wave: w, and w + NWV when there are more than NWV
  const int nrb = (RPW == 1) ? 1 : (w + NWV < NW ? 2 : 1);
  // stash: H pre-activation stacks per row block; a wave's second row block
  // is NWV blocks further
  float* stash_w = args.stash + (size_t)blockIdx.x * args.stash_per_wg + (size_t)w * H * NCB * 256;
  const size_t stash_rb = (size_t)NWV * H * NCB * 256;
  const uint32_t lo16 = (uint32_t)lane * 16u;   // this lane's byte offset in a 1 KiB wave fragment
  const float nu = args.nu;
  const bool prio = args.prio != 0;   // raise the younger waves' priority for their GEMMs
  constexpr bool SV = ACT == ACT_TANH;  // one-row-block kernels: the stash keeps tanh(z0)

  // segment accumulators; dW_{H+1} entry tid + r*nthr is thread tid's
  float lacc[6];
  float dwo[RPW], dbo = 0.f;
#pragma unroll
  for (int r = 0; r < RPW; ++r) dwo[r] = 0.f;

  // Item ranges: range blockIdx.x, or, with a counter, ranges taken in turn
  // until none is left (workgroups that share a compute unit do not progress
  // at the same rate, so a static split would leave the slower one last).
  int* s_range = reinterpret_cast<int*>(lds + L.sched);
  int range = blockIdx.x;
  for (;;) {
  if (args.counter) {
    __syncthreads();   // every thread has read the previous range index
    if (tid == 0) *s_range = atomicAdd(args.counter, 1);
    __syncthreads();
    range = *s_range;
  }
  if (range >= args.n_ranges) break;
  const int it0 = ((const CONST_AS int32_t*)args.wg_begin)[range];
  const int it1 = ((const CONST_AS int32_t*)args.wg_begin)[range + 1];
  for (int it = it0; it < it1; ++it) {
    __syncthreads();   // the previous tile's readers of xin/acc1 are done
    const CONST_AS Item& ir = ((const CONST_AS Item*)args.items)[it];
    Item item;
    item.sub = ir.sub;
    item.kind = ir.kind;
    item.start = ir.start;
    item.count = ir.count;
    item.slab = ir.slab;
    item.flags = ir.flags;
    const CONST_AS SubDev& sd = ((const CONST_AS SubDev*)args.subs)[item.sub];
    const float* fr = sd.frag;
    const float* W1p = fr + sh.f_w1;
    const float* bp = fr + sh.f_b;
    const float* Wop = fr + sh.f_wo;
    const float* bop = fr + sh.f_bo;
    const bool pde = item.kind == ITEM_PDE;

    if (item.flags & ITEM_FIRST) {
#pragma unroll
      for (int k = 0; k < 6; ++k) lacc[k] = 0.f;
#pragma unroll
      for (int r = 0; r < RPW; ++r) dwo[r] = 0.f;
      dbo = 0.f;
      for (int k = tid; k < Wp * D; k += nthr) acc1[k] = 0.f;
      for (int k = tid; k < H * Wp; k += nthr) dbacc[k] = 0.f;
    }

    // ---- stage the tile's input points into LDS
    if (pde) {
      for (int k = tid; k < MP::NPTS * D; k += nthr) {
        const int pt = k / D;
        xin[k] = (pt < item.count) ? ldg(sd.pde_x + (size_t)(item.start + pt) * D + (k - pt * D)) : 0.f;
      }
    } else {
      for (int k = tid; k < NCOL * D; k += nthr) {
        const int pt = k / D, q = k - pt * D;
        float v = 0.f;
        if (pt < item.count) {
          int idx = item.start + pt;
          if (idx < sd.n_obs) v = ldg(sd.obs_x + (size_t)idx * D + q);
          else if ((idx -= sd.n_obs) < sd.n_gh) v = ldg(sd.gh_x + (size_t)idx * D + q);
          else v = ldg(sd.anc_x + (size_t)(idx - sd.n_gh) * D + q);
        }
        xin[k] = v;
      }
    }
    __syncthreads();

    v4f acc[NCB];
    // ---- forward: input layer.  Activations ping-pong between the two LDS
    // stacks, so one barrier per layer suffices and each wave's activation
    // work overlaps the other waves' GEMMs.
    float* hin = bufH;
    float* hout = bufG;
    if constexpr (RPW == 1) {
      // The stash keeps each layer's pre-activation stack for the adjoint;
      // with tanh its value channel keeps tanh(z0) instead of z0 (the
      // adjoint needs z0 only through tanh and its derivatives, which are
      // polynomials in tanh), so the backward does not evaluate tanh again.
      const int nvb = pde ? MP::NPB : MV::NPB;   // value-channel column blocks
      auto stash_layer = [&](int li, bool value_blocks) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          if ((cb < nvb) == value_blocks || !SV) stg4u(stash_w + (li * NCB + cb) * 256, lo16, acc[cb]);
      };
      if (pde) input_layer_t<DIM, NCB, M_PDE>(acc, W1p, bp, xin, w, g, j);
      else input_layer_t<DIM, NCB, M_VALUE>(acc, W1p, bp, xin, w, g, j);
      stash_layer(0, false);
      if (pde) act_forward<DIM, NCB, M_PDE, ACT>(acc);
      else act_forward<DIM, NCB, M_VALUE, ACT>(acc);
      if constexpr (SV) stash_layer(0, true);
      store_fwd_t<NCB>(hin, S, acc, w, g, j);
      __syncthreads();

      // ---- forward: hidden layers 2..H
      for (int l = 2; l <= H; ++l) {
        const float* Wf = fr + sh.f_hid + (size_t)(l - 2) * 2 * Wp * Wp + (size_t)w * 16 * Wp;
        // The two waves sharing a SIMD run the same GEMM; the hardware favours
        // the older one, which then idles at the next barrier while the younger
        // finishes.  Raising the younger half's priority for the GEMM evens them.
        if (prio && w >= (NW >> 1)) __builtin_amdgcn_s_setprio(2);
        gemm_rows<NCB, true, true, DIM == 2>(Wf, hin, S, K4, g, j, lane, acc, KT);
        __builtin_amdgcn_s_setprio(0);
        if (pde) add_bias_t<NCB, MP::NPB>(acc, bp + (l - 1) * Wp, w, j);
        else add_bias_t<NCB, MV::NPB>(acc, bp + (l - 1) * Wp, w, j);
        stash_layer(l - 1, false);
        if (pde) act_forward<DIM, NCB, M_PDE, ACT>(acc);
        else act_forward<DIM, NCB, M_VALUE, ACT>(acc);
        if constexpr (SV) stash_layer(l - 1, true);
        store_fwd_t<NCB>(hout, S, acc, w, g, j);
        __syncthreads();
        float* t = hin;
        hin = hout;
        hout = t;
      }
    } else if constexpr (SPLIT) {
      // two row blocks per wave, one activation stack: every wave's GEMMs read
      // the stack before any wave overwrites it; the first block's
      // pre-activations wait in the stash meanwhile
      hin = bufG;
      for (int r = 0; r < nrb; ++r) {
        const int rb = w + r * NWV;
        float* st = stash_w + r * stash_rb;
        if (pde) input_layer<DIM, NCB, M_PDE>(acc, W1p, bp, xin, rb, g, j);
        else input_layer<DIM, NCB, M_VALUE>(acc, W1p, bp, xin, rb, g, j);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) stg4u(st + (0 * NCB + cb) * 256, lo16, acc[cb]);
        if (pde) act_forward<DIM, NCB, M_PDE, ACT>(acc);
        else act_forward<DIM, NCB, M_VALUE, ACT>(acc);
        store_fwd<NCB>(hin, S, acc, rb, g, j);
      }
      __syncthreads();
      for (int l = 2; l <= H; ++l) {
        const float* Wl = fr + sh.f_hid + (size_t)(l - 2) * 2 * Wp * Wp;
        for (int r = 0; r < nrb; ++r) {
          const int rb = w + r * NWV;
          float* st = stash_w + r * stash_rb;
          const float* Wf = Wl + (size_t)rb * 16 * Wp;
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc[cb] = zero4();
          if (prio && w >= (NWV >> 1)) __builtin_amdgcn_s_setprio(2);
          gemm_rows<NCB>(Wf, hin, S, K4, g, j, lane, acc, KT);
          __builtin_amdgcn_s_setprio(0);
          if (pde) add_bias<NCB, MP::NPB>(acc, bp + (l - 1) * Wp, rb, g);
          else add_bias<NCB, MV::NPB>(acc, bp + (l - 1) * Wp, rb, g);
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) stg4u(st + ((l - 1) * NCB + cb) * 256, lo16, acc[cb]);
        }
        __syncthreads();
        for (int r = nrb - 1; r >= 0; --r) {
          if (r != nrb - 1) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[cb] = ldg4u(stash_w + r * stash_rb + ((l - 1) * NCB + cb) * 256, lo16);
          }
          if (pde) act_forward<DIM, NCB, M_PDE, ACT>(acc);
          else act_forward<DIM, NCB, M_VALUE, ACT>(acc);
          store_fwd<NCB>(hin, S, acc, w + r * NWV, g, j);
        }
        __syncthreads();
      }
    } else {
      // two row blocks per wave: the same steps per row block
      for (int r = 0; r < nrb; ++r) {
        const int rb = w + r * NWV;
        float* st = stash_w + r * stash_rb;
        if (pde) input_layer<DIM, NCB, M_PDE>(acc, W1p, bp, xin, rb, g, j);
        else input_layer<DIM, NCB, M_VALUE>(acc, W1p, bp, xin, rb, g, j);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) stg4u(st + (0 * NCB + cb) * 256, lo16, acc[cb]);
        if (pde) act_forward<DIM, NCB, M_PDE, ACT>(acc);
        else act_forward<DIM, NCB, M_VALUE, ACT>(acc);
        store_fwd<NCB>(hin, S, acc, rb, g, j);
      }
      __syncthreads();
      for (int l = 2; l <= H; ++l) {
        const float* Wl = fr + sh.f_hid + (size_t)(l - 2) * 2 * Wp * Wp;
        for (int r = 0; r < (ks ? 1 : nrb); ++r) {
          const int rb = w + r * NWV;
          float* st = stash_w + r * stash_rb;
          const float* Wf = Wl + (size_t)rb * 16 * Wp;
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc[cb] = zero4();
          if (prio && w >= (NWV >> 1)) __builtin_amdgcn_s_setprio(2);
          gemm_rows<NCB>(Wf, hin, S, K4, g, j, lane, acc, KT);
          __builtin_amdgcn_s_setprio(0);
          if (pde) add_bias<NCB, MP::NPB>(acc, bp + (l - 1) * Wp, rb, g);
          else add_bias<NCB, MV::NPB>(acc, bp + (l - 1) * Wp, rb, g);
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) stg4u(st + ((l - 1) * NCB + cb) * 256, lo16, acc[cb]);
          if (pde) act_forward<DIM, NCB, M_PDE, ACT>(acc);
          else act_forward<DIM, NCB, M_VALUE, ACT>(acc);
          store_fwd<NCB>(hout, S, acc, rb, g, j);
        }
        if (ks) {
          // the two extra row blocks: half of the K range each for waves
          // 0..3 (block NWV + (w & 1), half w >> 1), summed by the owner
          if (w < 4) {
            const int e = NWV + (w & 1), c0 = (w >> 1) ? KCh / 2 : 0, c1 = (w >> 1) ? KCh : KCh / 2;
            gemm_rows_part<NCB>(Wl + (size_t)e * 16 * Wp, hin, S, KCh, KT, c0, c1, g, j, lane, acc);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) *reinterpret_cast<v4f*>(part + (w * NCB + cb) * 256 + lane * 4) = acc[cb];
          }
          __syncthreads();
          if (nrb == 2) {
            const int e = w + NWV;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              acc[cb] = *reinterpret_cast<const v4f*>(part + (w * NCB + cb) * 256 + lane * 4) +
                        *reinterpret_cast<const v4f*>(part + ((w + 2) * NCB + cb) * 256 + lane * 4);
            if (pde) add_bias<NCB, MP::NPB>(acc, bp + (l - 1) * Wp, e, g);
            else add_bias<NCB, MV::NPB>(acc, bp + (l - 1) * Wp, e, g);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) stg4u(stash_w + stash_rb + ((l - 1) * NCB + cb) * 256, lo16, acc[cb]);
            if (pde) act_forward<DIM, NCB, M_PDE, ACT>(acc);
            else act_forward<DIM, NCB, M_VALUE, ACT>(acc);
            store_fwd<NCB>(hout, S, acc, e, g, j);
          }
        }
        __syncthreads();
        float* t = hin;
        hin = hout;
        hout = t;
      }
    }

    // ---- output layer (h_H is in hin)
    if (pde) output_layer<DIM, NCB, M_PDE>(hin, S, Wp, Wop, bop, ys, tid, nthr);
    else output_layer<DIM, NCB, M_VALUE>(hin, S, Wp, Wop, bop, ys, tid, nthr);
    __syncthreads();

    // ---- residuals, losses and output seeds ybar = dL/dy
    if (pde) {
      if (tid < MP::NPTS) {
        const int pb = tid >> 4, jj = tid & 15;
        auto col = [&](int c) { return (c * MP::NPB + pb) * 16 + jj; };
        auto Y = [&](int c, int o) { return ys[o * NCOL + col(c)]; };
        float r[D];
        residuals<DIM>(Y, nu, r);
        const bool valid = tid < item.count;
        float sq = 0.f;
        float rb[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          if (!valid) r[k] = 0.f;
          sq += r[k] * r[k];
          rb[k] = 2.f * sd.lam[1] * sd.inv_n[0] * r[k];
        }
        lacc[1] += sq;
        // dL/dy for every channel (derivative of sum_k rb_k r_k / 2 ...)
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
          float s = 0.f;
#pragma unroll
          for (int k = 0; k < DIM; ++k) s += rb[k] * Y(1 + i, k);
          yb[i * NCOL + col(0)] = s;                              // u_i
#pragma unroll
          for (int jx = 0; jx < DIM; ++jx) {
            yb[i * NCOL + col(1 + jx)] = rb[i] * Y(0, jx) + (i == jx ? rb[DIM] : 0.f);   // d_j u_i
            yb[i * NCOL + col(DIM + 2 + jx)] = -nu * rb[i];                               // d_jj u_i
          }
          yb[i * NCOL + col(1 + DIM)] = rb[i];                     // d_t u_i
        }
        yb[DIM * NCOL + col(0)] = 0.f;                             // p
#pragma unroll
        for (int jx = 0; jx < DIM; ++jx) {
          yb[DIM * NCOL + col(1 + jx)] = rb[jx];                   // d_j p
          yb[DIM * NCOL + col(DIM + 2 + jx)] = 0.f;
        }
        yb[DIM * NCOL + col(1 + DIM)] = 0.f;
      }
    } else {
      // one column per point; a workgroup may have fewer threads than columns
      for (int col = tid; col < NCOL; col += nthr) {
        float e[D];
#pragma unroll
        for (int o = 0; o < D; ++o) e[o] = 0.f;
        if (col < item.count) {
          int idx = item.start + col;
          float y[D];
#pragma unroll
          for (int o = 0; o < D; ++o) y[o] = ys[o * NCOL + col];
          if (idx < sd.n_obs) {
            float sq = 0.f;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              const float d0 = y[i] - ldg(sd.obs_u + (size_t)idx * DIM + i);
              sq += sd.cw[i] * d0 * d0;
              e[i] = 2.f * sd.lam[0] * sd.inv_n[1] * sd.cw[i] * d0;
            }
            lacc[0] += sq;
          } else if ((idx -= sd.n_obs) < sd.n_gh) {
            float sq = 0.f;
            const float* tg = sd.gh_up + (size_t)idx * D;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              const float d0 = y[i] - tg[i];
              sq += sd.cw[i] * d0 * d0;
              e[i] = 2.f * sd.lam[2] * sd.inv_n[2] * sd.cw[i] * d0;
            }
            lacc[2] += sq;
            const float dp = y[DIM] - tg[DIM];
            if (sd.gh_kind[idx]) {
              lacc[4] += dp * dp;
              e[DIM] = 2.f * sd.lam[4] * sd.inv_n[2] * dp;
            } else {
              lacc[3] += dp * dp;
              e[DIM] = 2.f * sd.lam[3] * sd.inv_n[2] * dp;
            }
          } else {
            idx -= sd.n_gh;
            const float dp = y[DIM] - ldg(sd.anc_p + idx);
            lacc[5] += dp * dp;
            e[DIM] = 2.f * sd.lam[5] * sd.inv_n[3] * dp;
          }
        }
#pragma unroll
        for (int o = 0; o < D; ++o) yb[o * NCOL + col] = e[o];
      }
    }
    __syncthreads();

    if constexpr (RPW == 1) {
      // ---- output layer adjoint (z_H is fetched from the stash meanwhile)
      v4f zs[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        zs[cb] = ldg4u(stash_w + ((H - 1) * NCB + cb) * 256, lo16);
      {
        const int npb = pde ? MP::NPB : MV::NPB;
        if (tid < D * Wp) {
          const int o = tid / Wp, n = tid - o * Wp;
          float s = 0.f;
          for (int col = 0; col < NCOL; ++col) s += yb[o * NCOL + col] * hin[col * S + n];
          dwo[0] += s;
        }
        if (tid < D) {
          float s = 0.f;
          for (int col = 0; col < 16 * npb; ++col) s += yb[tid * NCOL + col];
          dbo += s;
        }
        {
          // lane (g, j): neuron 16w + j of columns 16cb + 4g + i (transposed tile)
          float wo[D];
#pragma unroll
          for (int o = 0; o < D; ++o) wo[o] = ldg(Wop + o * Wp + 16 * w + j);
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              float s = 0.f;
#pragma unroll
              for (int o = 0; o < D; ++o) s += wo[o] * yb[o * NCOL + 16 * cb + 4 * g + i];
              acc[cb][i] = s;
            }
        }
      }

      // ---- hidden and input layer adjoints (transposed tiles)
      for (int l = H; l >= 1; --l) {
        if (pde) act_adjoint<DIM, NCB, M_PDE, ACT, SV>(acc, zs);
        else act_adjoint<DIM, NCB, M_VALUE, ACT, SV>(acc, zs);
        // db_l: value-channel columns of this lane's neuron
        {
          const int npb = pde ? MP::NPB : MV::NPB;
          float s = 0.f;
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            if (cb < npb) s += (acc[cb][0] + acc[cb][1]) + (acc[cb][2] + acc[cb][3]);
          s = sum_groups(s);
          if (g == 0) dbacc[(l - 1) * Wp + 16 * w + j] += s;
        }
        if (l == 1) {
          // input layer: dW1[r][q] += sum_pts zbar0 xi_q + zbar_q (first-derivative channel q)
          const int r = 16 * w + j;
          float v[D];
#pragma unroll
          for (int q = 0; q < D; ++q) v[q] = 0.f;
          if (pde) {
#pragma unroll
            for (int pb = 0; pb < MP::NPB; ++pb)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const float* xp = xin + (16 * pb + 4 * g + i) * D;
#pragma unroll
                for (int q = 0; q < D; ++q)
                  v[q] += acc[pb][i] * xp[q] + acc[(1 + q) * MP::NPB + pb][i];
              }
          } else {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const float* xp = xin + (16 * cb + 4 * g + i) * D;
#pragma unroll
                for (int q = 0; q < D; ++q) v[q] += acc[cb][i] * xp[q];
              }
          }
#pragma unroll
          for (int q = 0; q < D; ++q) {
            const float s = sum_groups(v[q]);
            if (g == 0) acc1[r * D + q] += s;
          }
          break;
        }
        // z_{l-1} from the stash (kept for the next adjoint); then wait until
        // every wave has finished reading the LDS stacks before overwriting them
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          zs[cb] = ldg4u(stash_w + ((l - 2) * NCB + cb) * 256, lo16);
        __syncthreads();
        store_fwd_t<NCB>(bufG, S, acc, w, g, j);
        // recompute h_{l-1} from z_{l-1}
        if (pde) act_store_bwd_t<DIM, NCB, M_PDE, ACT, SV>(bufH, S2, zs, w, g, j);
        else act_store_bwd_t<DIM, NCB, M_VALUE, ACT, SV>(bufH, S2, zs, w, g, j);
        __syncthreads();
        // dW_l += Zbar_l H_{l-1}^T into this segment's slab, Zbar_l from the
        // registers (at most 8 column blocks: widths up to 128); the slab's
        // current values are requested before the GEMMs so the reads overlap them
        {
          float* sw = args.slabs + (size_t)item.slab * sh.slab_floats + sh.s_hid + (size_t)(l - 2) * Wp * Wp;
          const bool first = item.flags & ITEM_FIRST;
          if (prio && w >= (NW >> 1)) __builtin_amdgcn_s_setprio(2);   // as in the forward GEMM
          // the current slab values of both groups are requested up front
          v4f old8[8];
#pragma unroll
          for (int t = 0; t < 8; ++t)
            old8[t] = (t < NW && !first) ? ldg4u(sw + (size_t)(w * NW + t) * 256, lo16) : zero4();
          for (int nb0 = 0; nb0 < NW; nb0 += 4) {
            const int nnb = (NW - nb0) < 4 ? (NW - nb0) : 4;
            v4f old[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) old[t] = nb0 == 0 ? old8[t] : old8[4 + t];
            v4f dw[4] = {zero4(), zero4(), zero4(), zero4()};
            switch (nnb) {
              case 4: gemm_dw_t<NCB, 4>(acc, bufH, S2, g, j, nb0, dw); break;
              case 3: gemm_dw_t<NCB, 3>(acc, bufH, S2, g, j, nb0, dw); break;
              case 2: gemm_dw_t<NCB, 2>(acc, bufH, S2, g, j, nb0, dw); break;
              default: gemm_dw_t<NCB, 1>(acc, bufH, S2, g, j, nb0, dw); break;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (t < nnb) stg4u(sw + (size_t)(w * NW + nb0 + t) * 256, lo16, old[t] + dw[t]);
          }
        }
        __builtin_amdgcn_s_setprio(0);
        // Hbar_{l-1} = W_l^T Zbar_l
        {
          const float* WT = fr + sh.f_hid + (size_t)(l - 2) * 2 * Wp * Wp + (size_t)Wp * Wp + (size_t)w * 16 * Wp;
          if (prio && w >= (NW >> 1)) __builtin_amdgcn_s_setprio(2);
          gemm_rows<NCB, true, true, DIM == 2>(WT, bufG, S, K4, g, j, lane, acc, KT);
          __builtin_amdgcn_s_setprio(0);
        }
      }
    } else {
      // ---- two row blocks per wave (more than 8 row blocks): the same steps
      // per row block.  Only one block's zbar fits in registers across a
      // barrier, so the first block's waits in its own stash slot (z_l of
      // that block is dead once its adjoint has run).
      v4f zs[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        zs[cb] = ldg4u(stash_w + ((H - 1) * NCB + cb) * 256, lo16);
      {
        const int npb = pde ? MP::NPB : MV::NPB;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const int idx = tid + r * nthr;
          if (idx < D * Wp) {
            const int o = idx / Wp, n = idx - o * Wp;
            float s = 0.f;
            for (int col = 0; col < NCOL; ++col) s += yb[o * NCOL + col] * hin[col * S + n];
            dwo[r] += s;
          }
        }
        if (tid < D) {
          float s = 0.f;
          for (int col = 0; col < 16 * npb; ++col) s += yb[tid * NCOL + col];
          dbo += s;
        }
      }
      const bool raise = prio && w >= (NWV >> 1);   // wave priority for the GEMMs, as in the forward
      for (int r = 0; r < nrb; ++r) {
        const int rb = w + r * NWV;
        float* st = stash_w + r * stash_rb;
        if (r > 0) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) zs[cb] = ldg4u(st + ((H - 1) * NCB + cb) * 256, lo16);
        }
        out_adjoint_rows<D, NCB>(acc, Wop, yb, Wp, rb, g, j);
        if (pde) adjoint_rows<DIM, NCB, M_PDE, ACT>(acc, zs, dbacc, acc1, xin, Wp, rb, H, g, j);
        else adjoint_rows<DIM, NCB, M_VALUE, ACT>(acc, zs, dbacc, acc1, xin, Wp, rb, H, g, j);
        if (H > 1 && (SPLIT || r + 1 < nrb)) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) stg4u(st + ((H - 1) * NCB + cb) * 256, lo16, acc[cb]);
        }
      }
      if constexpr (SPLIT) {
        // The tile's columns in two halves (Zbar and H_{l-1} of one half fit
        // in LDS at a time; the GEMMs are separable over columns).  Every
        // block's zbar and hbar wait in its own stash slot between barriers.
        constexpr int NCBH = NCB / 2;
        for (int l = H; l >= 2; --l) {
          float* sw = args.slabs + (size_t)item.slab * sh.slab_floats + sh.s_hid + (size_t)(l - 2) * Wp * Wp;
          const size_t zl = (size_t)(l - 1) * NCB * 256, zp = (size_t)(l - 2) * NCB * 256;
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            // this half's Zbar_l of both row blocks: the wave's own stash
            // slots, so they are requested before the barrier (which only
            // guards the LDS stacks)
            v4f t[NCBH];
            v4f tz[2][NCBH];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
              if (r < nrb) {
#pragma unroll
                for (int c = 0; c < NCBH; ++c)
                  tz[r][c] = ldg4u(stash_w + r * stash_rb + zl + ((size_t)hh * NCBH + c) * 256, lo16);
              }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 2; ++r)
              if (r < nrb) store_fwd<NCBH>(bufG, S, tz[r], w + r * NWV, g, j);
            // H_{l-1} of this half, recomputed from z_{l-1}
            for (int r = 0; r < nrb; ++r) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) zs[cb] = ldg4u(stash_w + r * stash_rb + zp + cb * 256, lo16);
              if (hh == 0) {
                if (pde) act_store_bwd_cols<DIM, NCB, M_PDE, ACT, 0, NCBH>(bufH, S2, zs, w + r * NWV, g, j);
                else act_store_bwd_cols<DIM, NCB, M_VALUE, ACT, 0, NCBH>(bufH, S2, zs, w + r * NWV, g, j);
              } else {
                if (pde) act_store_bwd_cols<DIM, NCB, M_PDE, ACT, NCBH, NCBH>(bufH, S2, zs, w + r * NWV, g, j);
                else act_store_bwd_cols<DIM, NCB, M_VALUE, ACT, NCBH, NCBH>(bufH, S2, zs, w + r * NWV, g, j);
              }
            }
            __syncthreads();
            if (raise) __builtin_amdgcn_s_setprio(2);
            dw_tiles<NCBH>(sw, (item.flags & ITEM_FIRST) && hh == 0, bufG, S, bufH, S2, NW, dw_t0, dw_t1, g, j,
                           lo16);
            // Hbar_{l-1} of this half into the stash slot of Zbar_l (consumed)
            const float* WTl = fr + sh.f_hid + (size_t)(l - 2) * 2 * Wp * Wp + (size_t)Wp * Wp;
            for (int r = 0; r < nrb; ++r) {
              const int rb = w + r * NWV;
#pragma unroll
              for (int c = 0; c < NCBH; ++c) t[c] = zero4();
              const float* WT = WTl + (size_t)rb * 16 * Wp;
              gemm_rows<NCBH>(WT, bufG, S, K4, g, j, lane, t, KT);
              float* st = stash_w + r * stash_rb + zl + (size_t)hh * NCBH * 256;
#pragma unroll
              for (int c = 0; c < NCBH; ++c) stg4u(st + c * 256, lo16, t[c]);
            }
            __builtin_amdgcn_s_setprio(0);
          }
          // adjoint of layer l-1 per block; zbar_{l-1} replaces z_{l-1}
          for (int r = 0; r < nrb; ++r) {
            const int rb = w + r * NWV;
            float* st = stash_w + r * stash_rb;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[cb] = ldg4u(st + zl + cb * 256, lo16);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) zs[cb] = ldg4u(st + zp + cb * 256, lo16);
            if (pde) adjoint_rows<DIM, NCB, M_PDE, ACT>(acc, zs, dbacc, acc1, xin, Wp, rb, l - 1, g, j);
            else adjoint_rows<DIM, NCB, M_VALUE, ACT>(acc, zs, dbacc, acc1, xin, Wp, rb, l - 1, g, j);
            if (l > 2) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) stg4u(st + zp + cb * 256, lo16, acc[cb]);
            }
          }
        }
      } else {
        // every block's Zbar_l and H_{l-1} fit in LDS together
        for (int l = H; l >= 2; --l) {
          // the first block's Zbar_l and z_{l-1} come from the wave's own
          // stash slots: in 2D they are requested before the barrier (which
          // only guards the LDS stacks), so their latency overlaps the wait
          // (the 3D kernels have no registers to hold them across it)
          constexpr bool early = DIM == 2;
          v4f zb[NCB];
          if (early) {
            if (nrb == 2) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) zb[cb] = ldg4u(stash_w + ((l - 1) * NCB + cb) * 256, lo16);
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) zs[cb] = ldg4u(stash_w + ((l - 2) * NCB + cb) * 256, lo16);
          }
          __syncthreads();
          // Zbar_l into LDS: the last block's from registers, the first's from the stash
          store_fwd<NCB>(bufG, S, acc, w + (nrb - 1) * NWV, g, j);
          if (nrb == 2) {
            if (!early) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) zb[cb] = ldg4u(stash_w + ((l - 1) * NCB + cb) * 256, lo16);
            }
            store_fwd<NCB>(bufG, S, zb, w, g, j);
          }
          // h_{l-1} recomputed from z_{l-1}
          for (int r = 0; r < nrb; ++r) {
            if (r > 0 || !early) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb)
                zs[cb] = ldg4u(stash_w + r * stash_rb + ((l - 2) * NCB + cb) * 256, lo16);
            }
            if (pde) act_store_bwd<DIM, NCB, M_PDE, ACT>(bufH, S2, zs, w + r * NWV, g, j);
            else act_store_bwd<DIM, NCB, M_VALUE, ACT>(bufH, S2, zs, w + r * NWV, g, j);
          }
          __syncthreads();
          float* sw = args.slabs + (size_t)item.slab * sh.slab_floats + sh.s_hid + (size_t)(l - 2) * Wp * Wp;
          if (raise) __builtin_amdgcn_s_setprio(2);
          dw_tiles<NCB>(sw, item.flags & ITEM_FIRST, bufG, S, bufH, S2, NW, dw_t0, dw_t1, g, j, lo16);
          __builtin_amdgcn_s_setprio(0);
          // Hbar_{l-1} = W_l^T Zbar_l, then the adjoint of layer l-1, per block
          const float* WTl = fr + sh.f_hid + (size_t)(l - 2) * 2 * Wp * Wp + (size_t)Wp * Wp;
          if (ks && w < 4) {
            // the extra row blocks' Hbar over half of the K range (as in the forward)
            const int e = NWV + (w & 1), c0 = (w >> 1) ? KCh / 2 : 0, c1 = (w >> 1) ? KCh : KCh / 2;
            if (raise) __builtin_amdgcn_s_setprio(2);
            gemm_rows_part<NCB>(WTl + (size_t)e * 16 * Wp, bufG, S, KCh, KT, c0, c1, g, j, lane, acc);
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) *reinterpret_cast<v4f*>(part + (w * NCB + cb) * 256 + lane * 4) = acc[cb];
          }
          for (int r = 0; r < (ks ? 1 : nrb); ++r) {
            const int rb = w + r * NWV;
            float* st = stash_w + r * stash_rb;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) zs[cb] = ldg4u(st + ((l - 2) * NCB + cb) * 256, lo16);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[cb] = zero4();
            const float* WT = WTl + (size_t)rb * 16 * Wp;
            if (raise) __builtin_amdgcn_s_setprio(2);
            gemm_rows<NCB>(WT, bufG, S, K4, g, j, lane, acc, KT);
            __builtin_amdgcn_s_setprio(0);
            if (pde) adjoint_rows<DIM, NCB, M_PDE, ACT>(acc, zs, dbacc, acc1, xin, Wp, rb, l - 1, g, j);
            else adjoint_rows<DIM, NCB, M_VALUE, ACT>(acc, zs, dbacc, acc1, xin, Wp, rb, l - 1, g, j);
            if (l > 2 && r + 1 < nrb) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) stg4u(st + ((l - 2) * NCB + cb) * 256, lo16, acc[cb]);
            }
          }
          if (ks) {
            if (nrb == 2) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) zs[cb] = ldg4u(stash_w + stash_rb + ((l - 2) * NCB + cb) * 256, lo16);
            }
            __syncthreads();   // the halves are in LDS
            if (nrb == 2) {
              const int e = w + NWV;
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb)
                acc[cb] = *reinterpret_cast<const v4f*>(part + (w * NCB + cb) * 256 + lane * 4) +
                          *reinterpret_cast<const v4f*>(part + ((w + 2) * NCB + cb) * 256 + lane * 4);
              if (pde) adjoint_rows<DIM, NCB, M_PDE, ACT>(acc, zs, dbacc, acc1, xin, Wp, e, l - 1, g, j);
              else adjoint_rows<DIM, NCB, M_VALUE, ACT>(acc, zs, dbacc, acc1, xin, Wp, e, l - 1, g, j);
            }
          }
        }
      }
    }

    // ---- end of segment: write the accumulated gradient pieces and losses
    if (item.flags & ITEM_LAST) {
      __syncthreads();
      float* slab = args.slabs + (size_t)item.slab * sh.slab_floats;
      for (int k = tid; k < Wp * D; k += nthr) slab[sh.s_w1 + k] = acc1[k];
      for (int k = tid; k < H * Wp; k += nthr) slab[sh.s_b + k] = dbacc[k];
#pragma unroll
      for (int r = 0; r < RPW; ++r)
        if (tid + r * nthr < D * Wp) slab[sh.s_wo + tid + r * nthr] = dwo[r];
      if (tid < 4) slab[sh.s_bo + tid] = (tid < D) ? dbo : 0.f;
      // loss partials: wave sums, then across waves
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        float v = lacc[k];
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[w * 8 + k] = v;
      }
      __syncthreads();
      if (tid < 8) {
        float v = 0.f;
        if (tid < 6)
          for (int q = 0; q < NWV; ++q) v += red[q * 8 + tid];
        slab[sh.s_loss + tid] = v;
      }
      __syncthreads();
    }
  }
  if (!args.counter) break;
  }
}

// ---------------------------------------------------------------------------
// Hidden-neuron positions.  A hidden layer's Wp positions are read by the four
// lane groups of a GEMM's K dimension in segments of Wp/4.  Neuron n sits at
// position (n / Kq) * (Wp/4) + n % Kq with Kq = ceil(W/4): the padding fills
// the tail of every segment, so the GEMMs stop after Kq K-steps instead of
// Wp/4.  This is a permutation of the hidden neurons with zero weights at the
// padded positions (whose activations are 0), so the network is unchanged.
// ---------------------------------------------------------------------------
__host__ __device__ inline int hid_pos(const Shape& sh, int n) { return (n / sh.Kq) * (sh.Wp / 4) + n % sh.Kq; }
__host__ __device__ inline int hid_neuron(const Shape& sh, int p) {
  const int seg = sh.Wp / 4, g = p / seg, s = p - g * seg, n = g * sh.Kq + s;
  return (s < sh.Kq && n < sh.W) ? n : -1;
}

// ---------------------------------------------------------------------------
// prep: fragment-ordered copies of the weights (hidden neurons at their
// positions, zeros at padded positions)
// ---------------------------------------------------------------------------
__global__ void prep_kernel(const PrepArgs a) {
  const Shape& sh = a.sh;
  const int s = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0 && idx < a.n_counters) a.counters[idx] = 0;
  if (idx >= sh.frag_floats) return;
  const float* th = a.subs[s].theta;
  float* fr = a.subs[s].frag;
  const int W = sh.W, Wp = sh.Wp, D = sh.D, H = sh.H;
  float v = 0.f;
  if (idx < sh.f_w1) {
    const int64_t per = 2LL * Wp * Wp;
    const int l = 2 + (int)(idx / per);
    const int64_t rem = idx - (int64_t)(l - 2) * per;
    const bool trans = rem >= (int64_t)Wp * Wp;
    const int e = (int)(trans ? rem - (int64_t)Wp * Wp : rem);
    const int q = e & 3, lane = (e >> 2) & 63, t = e >> 8;
    const int K4 = Wp / 16;
    const int s4 = t % K4, w = t / K4;
    const int k = hid_neuron(sh, (lane >> 4) * (Wp / 4) + 4 * s4 + q);
    const int r = hid_neuron(sh, 16 * w + (lane & 15));
    if (r >= 0 && k >= 0) v = trans ? th[sh.p_w[l] + (int64_t)k * W + r] : th[sh.p_w[l] + (int64_t)r * W + k];
  } else if (idx < sh.f_b) {
    const int e = (int)(idx - sh.f_w1), p = e / D, q = e - p * D, r = hid_neuron(sh, p);
    if (r >= 0) v = th[sh.p_w[1] + (int64_t)r * D + q];
  } else if (idx < sh.f_wo) {
    const int e = (int)(idx - sh.f_b), l = 1 + e / Wp, r = hid_neuron(sh, e % Wp);
    if (r >= 0) v = th[sh.p_b[l] + r];
  } else if (idx < sh.f_bo) {
    const int e = (int)(idx - sh.f_wo), o = e / Wp, n = hid_neuron(sh, e % Wp);
    if (n >= 0) v = th[sh.p_w[H + 1] + (int64_t)o * W + n];
  } else if (idx < sh.f_bo + 4) {
    const int o = (int)(idx - sh.f_bo);
    if (o < D) v = th[sh.p_b[H + 1] + o];
  }
  fr[idx] = v;
}

// ---------------------------------------------------------------------------
// reduce + Adam: sum this subdomain's slabs in a fixed order; Adam in place
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t slab_pos(const Shape& sh, int64_t p) {
  const int W = sh.W, Wp = sh.Wp, D = sh.D, H = sh.H;
  if (p < sh.p_b[1]) {                        // W1 [W][D]
    const int64_t r = p / D, q = p - r * D;
    return sh.s_w1 + (int64_t)hid_pos(sh, (int)r) * D + q;
  }
  if (p < sh.p_w[2 <= H ? 2 : H + 1]) {       // b1
    return sh.s_b + hid_pos(sh, (int)(p - sh.p_b[1]));
  }
  for (int l = 2; l <= H; ++l) {
    if (p < sh.p_b[l]) {                      // W_l [W][W] in accumulator order
      const int64_t e = p - sh.p_w[l];
      const int r0 = (int)(e / W), c0 = (int)(e - (int64_t)r0 * W);
      const int r = hid_pos(sh, r0), c = hid_pos(sh, c0);
      const int w = r >> 4, g = (r & 15) >> 2, i = r & 3, nb = c >> 4, jj = c & 15;
      return sh.s_hid + (int64_t)(l - 2) * Wp * Wp + ((int64_t)(w * sh.NW + nb) * 64 + g * 16 + jj) * 4 + i;
    }
    if (p < sh.p_w[l + 1]) return sh.s_b + (int64_t)(l - 1) * Wp + hid_pos(sh, (int)(p - sh.p_b[l]));
  }
  if (p < sh.p_b[H + 1]) {                    // W_{H+1} [D][W]
    const int64_t e = p - sh.p_w[H + 1];
    const int o = (int)(e / W), n = (int)(e - (int64_t)o * W);
    return sh.s_wo + (int64_t)o * Wp + hid_pos(sh, n);
  }
  return sh.s_bo + (p - sh.p_b[H + 1]);
}

// stage 1: partial[s][c][pos] = sum of slabs k0 + c*CH .. of subdomain s at
// position pos (consecutive threads read consecutive floats of each slab)
__global__ void slab_sum_kernel(const ReduceArgs a) {
  const Shape& sh = a.sh;
  const int s = blockIdx.y, c = blockIdx.z;
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= sh.slab_floats) return;
  const int k0 = a.seg_begin[s] + c * kSlabChunk;
  const int k1 = min(a.seg_begin[s + 1], k0 + kSlabChunk);
  float v[kSlabChunk];
#pragma unroll
  for (int q = 0; q < kSlabChunk; ++q)
    v[q] = (k0 + q < k1) ? a.slabs[(size_t)(k0 + q) * sh.slab_floats + pos] : 0.f;
  float acc = 0.f;
#pragma unroll
  for (int q = 0; q < kSlabChunk; ++q) acc += v[q];
  a.partial[((size_t)s * a.n_chunks + c) * sh.slab_floats + pos] = acc;
}

// stage 2: gradient of every parameter (partials in chunk order), its
// per-block sum of squares (for clipping), and the losses
__global__ void grad_kernel(const ReduceArgs a) {
  const Shape& sh = a.sh;
  const int s = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nseg = a.seg_begin[s + 1] - a.seg_begin[s];
  const int nc = (nseg + kSlabChunk - 1) / kSlabChunk;
  const float* part = a.partial + (size_t)s * a.n_chunks * sh.slab_floats;
  const SubDev& sd = a.subs[s];
  __shared__ float red[256];
  float g = 0.f;
  if (p < sh.P) {
    const int64_t pos = slab_pos(sh, p);
    for (int c = 0; c < nc; ++c) g += part[(size_t)c * sh.slab_floats + pos];
    a.gbuf[(size_t)s * sh.P + p] = g;
    if (a.grad_out) a.grad_out[(size_t)s * sh.P + p] = g;
  }
  red[threadIdx.x] = g * g;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.normpart[(size_t)s * gridDim.x + blockIdx.x] = red[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float L[7];
    for (int q = 0; q < 6; ++q) {
      float v = 0.f;
      for (int c = 0; c < nc; ++c) v += part[(size_t)c * sh.slab_floats + sh.s_loss + q];
      L[q] = v;
    }
    L[0] *= sd.inv_n[1];
    L[1] *= sd.inv_n[0];
    L[2] *= sd.inv_n[2];
    L[3] *= sd.inv_n[2];
    L[4] *= sd.inv_n[2];
    L[5] *= sd.inv_n[3];
    L[6] = sd.lam[0] * L[0] + sd.lam[1] * L[1] + sd.lam[2] * L[2] + sd.lam[3] * L[3] +
           sd.lam[4] * L[4] + sd.lam[5] * L[5];
    for (int q = 0; q < 7; ++q) {
      a.loss_ws[s * 8 + q] = L[q];
      if (a.loss_out) a.loss_out[s * 7 + q] = L[q];
    }
    a.loss_ws[s * 8 + 7] = 0.f;
  }
}

// global-norm clipping factor of each subdomain: min(1, c / ||g||), block
// sums added in a fixed order
__global__ void clip_kernel(const ReduceArgs a, int nblk) {
  const int s = blockIdx.x;
  __shared__ float red[256];
  float v = 0.f;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) v += a.normpart[(size_t)s * nblk + k];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float nrm = sqrtf(red[0]);
    a.clip_scale[s] = (a.clip > 0.f && nrm > a.clip) ? a.clip / nrm : 1.f;
  }
}

// stage 3: Adam on the (clipped) gradient, in place on theta, m, v
__global__ void adam_kernel(const ReduceArgs a) {
  const Shape& sh = a.sh;
  const int s = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!a.update || p >= sh.P) return;
  const SubDev& sd = a.subs[s];
  const float g = a.gbuf[(size_t)s * sh.P + p] * (a.clip > 0.f ? a.clip_scale[s] : 1.f);
  const float m = a.beta1 * sd.m[p] + (1.f - a.beta1) * g;
  const float v = a.beta2 * sd.v[p] + (1.f - a.beta2) * g * g;
  sd.m[p] = m;
  sd.v[p] = v;
  const float c1 = 1.f - powf(a.beta1, (float)a.t);
  const float c2 = 1.f - powf(a.beta2, (float)a.t);
  float* th = const_cast<float*>(sd.theta);
  th[p] = th[p] - a.lr * (m / c1) / (sqrtf(v / c2) + a.eps);
}

// ---------------------------------------------------------------------------
// query: routing (bin points by subdomain box) and grouped forward
// ---------------------------------------------------------------------------
__global__ void route_zero_kernel(int32_t* counts, int32_t* cursor, int n_sub) {
  for (int s = threadIdx.x; s < n_sub; s += blockDim.x) { counts[s] = 0; cursor[s] = 0; }
}

// Routing is a counting sort by subdomain.  Points are counted in a per-block
// LDS histogram and each block adds its counts to the global ones with one
// atomic per subdomain; the scatter reserves a contiguous slot range per
// (block, subdomain) the same way.  (Global atomics per point serialise on
// the few subdomain counters.)
constexpr int kRouteBlock = 256;

__device__ __forceinline__ int route_point(const RouteArgs& a, int64_t i) {
  const float* x = a.x + i * a.D;
  for (int s = 0; s < a.n_sub; ++s) {
    const float* lo = a.boxes + s * 8;
    const float* hi = lo + 4;
    bool in = true;
    for (int q = 0; q < a.D; ++q) {
      const float c = x[q];
      const bool ok = (c >= lo[q]) && (c < hi[q] || (c == hi[q] && hi[q] == a.gmax[q]));
      if (!ok) { in = false; break; }
    }
    if (in) return s;
  }
  return -1;
}

__global__ __launch_bounds__(kRouteBlock) void route_count_kernel(const RouteArgs a) {
  extern __shared__ int hist[];   // [n_sub]
  for (int s = threadIdx.x; s < a.n_sub; s += blockDim.x) hist[s] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n) {
    const int found = route_point(a, i);
    a.sub_id[i] = found;
    if (found >= 0) atomicAdd(&hist[found], 1);
    else
      for (int q = 0; q < a.out_cols; ++q) a.out[i * a.out_cols + q] = __builtin_nanf("");
  }
  __syncthreads();
  for (int s = threadIdx.x; s < a.n_sub; s += blockDim.x)
    if (hist[s]) atomicAdd(a.counts + s, hist[s]);
}

__global__ void route_offsets_kernel(const RouteArgs a) {
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int s = 0; s < a.n_sub; ++s) { a.offsets[s] = acc; acc += a.counts[s]; }
    a.offsets[a.n_sub] = acc;
  }
}

__global__ __launch_bounds__(kRouteBlock) void route_scatter_kernel(const RouteArgs a) {
  extern __shared__ int sh[];   // hist[n_sub], base[n_sub]
  int* hist = sh;
  int* base = sh + a.n_sub;
  for (int s = threadIdx.x; s < a.n_sub; s += blockDim.x) hist[s] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = (i < a.n) ? a.sub_id[i] : -1;
  const int rank = (s >= 0) ? atomicAdd(&hist[s], 1) : 0;
  __syncthreads();
  for (int q = threadIdx.x; q < a.n_sub; q += blockDim.x)
    base[q] = hist[q] ? a.offsets[q] + atomicAdd(a.cursor + q, hist[q]) : 0;
  __syncthreads();
  if (s >= 0) a.perm[base[s] + rank] = (int32_t)i;
}

// A small query routed by one workgroup: subdomain of every point, counts,
// offsets and the permutation from one launch instead of four.  Each thread
// keeps the subdomains of its points in registers between the two passes.
constexpr int kRouteSmallThreads = 1024;
constexpr int kRouteSmallPerThread = 8;
constexpr int kRouteSmallMax = kRouteSmallThreads * kRouteSmallPerThread;   // points

__global__ __launch_bounds__(kRouteSmallThreads) void route_small_kernel(const RouteArgs a) {
  extern __shared__ int sh[];   // hist[n_sub], base[n_sub]
  int* hist = sh;
  int* base = sh + a.n_sub;
  for (int s = threadIdx.x; s < a.n_sub; s += blockDim.x) hist[s] = 0;
  __syncthreads();
  int sid[kRouteSmallPerThread];
#pragma unroll
  for (int k = 0; k < kRouteSmallPerThread; ++k) {
    const int64_t i = threadIdx.x + (int64_t)k * kRouteSmallThreads;
    sid[k] = -1;
    if (i < a.n) {
      const int found = route_point(a, i);
      sid[k] = found;
      a.sub_id[i] = found;
      if (found >= 0) atomicAdd(&hist[found], 1);
      else
        for (int q = 0; q < a.out_cols; ++q) a.out[i * a.out_cols + q] = __builtin_nanf("");
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int s = 0; s < a.n_sub; ++s) {
      base[s] = acc;
      a.offsets[s] = acc;
      a.counts[s] = hist[s];
      acc += hist[s];
    }
    a.offsets[a.n_sub] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRouteSmallPerThread; ++k)
    if (sid[k] >= 0) a.perm[atomicAdd(&base[sid[k]], 1)] = (int32_t)(threadIdx.x + k * kRouteSmallThreads);
}

struct QueryLds { int S, NCOL, bufH, ys, xin, pidx, total; };
__host__ __device__ inline QueryLds query_lds(int D, int Wp, int NCB) {
  QueryLds L;
  L.NCOL = 16 * NCB;
  L.S = Wp + 4;
  int o = 0;
  L.bufH = o; o += (L.NCOL * L.S + 3) & ~3;
  L.ys = o;   o += (D * L.NCOL + 3) & ~3;
  L.xin = o;  o += (L.NCOL * D + 3) & ~3;
  L.pidx = o; o += L.NCOL;
  L.total = o;
  return L;
}

// forward of one staged tile (points in xin) through all layers; output in ys.
// Wave w computes row block w and, with RPW = 2, row block w + NWV; one LDS
// stack, so every block's accumulators wait in registers until all waves have
// read the stack.
template <int DIM, int NCB, int MODE, int ACT, int RPW>
__device__ __forceinline__ void forward_tile(const Shape& sh, const float* fr, float* bufH, float* ys,
                                             const float* xin, int S, int tid, int nthr, int w, int g,
                                             int j, int lane) {
  using M = ModeCfg<DIM, NCB, MODE>;
  const int Wp = sh.Wp, H = sh.H, K4 = sh.Kq >> 2, KT = sh.Kq & 3, NWV = sh.NWV;
  const int nrb = (RPW == 1) ? 1 : (w + NWV < sh.NW ? 2 : 1);
  v4f acc[RPW][NCB];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    if (r >= nrb) break;
    input_layer<DIM, NCB, MODE>(acc[r], fr + sh.f_w1, fr + sh.f_b, xin, w + r * NWV, g, j);
    act_forward<DIM, NCB, MODE, ACT>(acc[r]);
    store_fwd<NCB>(bufH, S, acc[r], w + r * NWV, g, j);
  }
  __syncthreads();
  for (int l = 2; l <= H; ++l) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      if (r >= nrb) break;
      const int rb = w + r * NWV;
      const float* Wf = fr + sh.f_hid + (size_t)(l - 2) * 2 * Wp * Wp + (size_t)rb * 16 * Wp;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[r][cb] = zero4();
      gemm_rows<NCB, false, false, RPW == 1>(Wf, bufH, S, K4, g, j, lane, acc[r], KT);
      add_bias<NCB, M::NPB>(acc[r], fr + sh.f_b + (l - 1) * Wp, rb, g);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      if (r >= nrb) break;
      act_forward<DIM, NCB, MODE, ACT>(acc[r]);
      store_fwd<NCB>(bufH, S, acc[r], w + r * NWV, g, j);
    }
    __syncthreads();
  }
  output_layer<DIM, NCB, MODE>(bufH, S, Wp, fr + sh.f_wo, fr + sh.f_bo, ys, tid, nthr);
  __syncthreads();
}

// SMALL: one 16-point block per channel of the mode instead of CF column
// blocks, which halves (gradient mode) or divides by six (value mode) the
// work on a tile's critical path; for requests too small to fill the chip.
template <int DIM, int MODE, int ACT, int RPW, int SMALL>
__global__ __launch_bounds__(512) void query_kernel(const QueryArgs a) {
  constexpr int D = DIM + 1, CF = 2 * DIM + 2;
  constexpr int CMODE = MODE == M_VALUE ? 1 : (MODE == M_GRAD ? DIM + 1 : CF);
  constexpr int NCB = SMALL ? CMODE : CF;
  using M = ModeCfg<DIM, NCB, MODE>;
  constexpr int NPTS = M::NPTS, NCOL = 16 * NCB;
  extern __shared__ float lds[];
  const Shape& sh = a.sh;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, g = lane >> 4, j = lane & 15;
  const QueryLds L = query_lds(D, sh.Wp, NCB);
  float* bufH = lds + L.bufH;
  float* ys = lds + L.ys;
  float* xin = lds + L.xin;
  int32_t* pidx = reinterpret_cast<int32_t*>(lds + L.pidx);

  // tiles: for routed queries, subdomain s holds points [offsets[s], offsets[s]+counts[s])
  const int nsub = a.counts ? a.n_sub : 1;
  int64_t total = 0;
  for (int s = 0; s < nsub; ++s) {
    const int64_t c = a.counts ? a.counts[s] : a.n;
    total += (c + NPTS - 1) / NPTS;
  }
  // Tiles are ordered by subdomain.  Workgroups are dispatched to the eight
  // XCDs round-robin (workgroup b on XCD b mod 8), each XCD with its own L2:
  // with a grid that is a multiple of 8, XCD x takes the x-th eighth of the
  // tiles, so each L2 holds the weights of a few subdomains, not all.
  int64_t t0 = blockIdx.x, tend = total, tstep = gridDim.x;
  if (gridDim.x >= 16 && (gridDim.x & 7) == 0) {
    const int64_t x = blockIdx.x & 7;
    t0 = x * total / 8 + (blockIdx.x >> 3);
    tend = (x + 1) * total / 8;
    tstep = gridDim.x >> 3;
  }
  for (int64_t t = t0; t < tend; t += tstep) {
    int s = 0;
    int64_t tl = t, c = 0;
    for (; s < nsub; ++s) {
      c = a.counts ? a.counts[s] : a.n;
      const int64_t nt = (c + NPTS - 1) / NPTS;
      if (tl < nt) break;
      tl -= nt;
    }
    const int sub = a.counts ? s : a.sub;
    const int64_t base = (a.counts ? a.offsets[s] : 0) + tl * NPTS;
    const int cnt = (int)((c - tl * NPTS) < NPTS ? (c - tl * NPTS) : NPTS);
    for (int k = tid; k < NPTS; k += nthr)
      pidx[k] = (k < cnt) ? (a.perm ? a.perm[base + k] : (int32_t)(base + k)) : -1;
    __syncthreads();
    for (int k = tid; k < NCOL * D; k += nthr) {
      const int pt = k / D;
      float v = 0.f;
      if (pt < NPTS && pidx[pt] >= 0) v = a.x[(size_t)pidx[pt] * D + (k - pt * D)];
      xin[k] = v;
    }
    __syncthreads();
    forward_tile<DIM, NCB, MODE, ACT, RPW>(sh, a.subs[sub].frag, bufH, ys, xin, L.S, tid, nthr, w, g, j, lane);
    for (int k = tid; k < NPTS; k += nthr) {
      if (pidx[k] < 0) continue;
      const int64_t q = pidx[k];
      const int pb = k >> 4, jj = k & 15;
      auto Y = [&](int ch, int o) { return ys[o * NCOL + (ch * M::NPB + pb) * 16 + jj]; };
      if (a.what == Q_VALUE) {
        for (int o = 0; o < D; ++o) a.out[q * D + o] = Y(0, o);
      } else if (a.what == Q_UVPW) {
        if constexpr (MODE == M_GRAD && DIM == 2) {
          a.out[q * 4 + 0] = Y(0, 0);
          a.out[q * 4 + 1] = Y(0, 1);
          a.out[q * 4 + 2] = Y(0, 2);
          a.out[q * 4 + 3] = Y(1, 1) - Y(2, 0);   // v_x - u_y
        }
      } else if (a.what == Q_CHANNELS) {
        if constexpr (MODE == M_PDE)
          for (int ch = 0; ch < CF; ++ch)
            for (int o = 0; o < D; ++o) a.out[(q * CF + ch) * D + o] = Y(ch, o);
      } else {
        if constexpr (MODE == M_PDE) {
          float r[D];
          residuals<DIM>(Y, a.nu, r);
          for (int k = 0; k < D; ++k) a.out[q * D + k] = r[k];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// exchange: neighbour values at ghost points, anchor-normalised pressure
// ---------------------------------------------------------------------------
template <int DIM, int ACT, int RPW>
__global__ __launch_bounds__(512) void exchange_kernel(const ExchangeArgs a) {
  constexpr int D = DIM + 1, CF = 2 * DIM + 2, NCB = CF, NCOL = 16 * NCB;
  extern __shared__ float lds[];
  const Shape& sh = a.sh;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, g = lane >> 4, j = lane & 15;
  const QueryLds L = query_lds(D, sh.Wp, NCB);
  float* bufH = lds + L.bufH;
  float* ys = lds + L.ys;
  float* xin = lds + L.xin;
  for (int t = blockIdx.x; t < a.n_items; t += gridDim.x) {
    const ExchangeItem it = a.items[t];
    const SubDev& ra = a.subs[it.a];
    const int half = NCOL / 2;
    for (int k = tid; k < NCOL * D; k += nthr) {
      const int pt = k / D, q = k - pt * D;
      float v = 0.f;
      if (it.paired) {
        const int pp = pt < half ? pt : pt - half;
        if (pp < it.count) {
          const float* gx = ra.gh_x + (size_t)(it.start + pp) * D;
          v = (pt < half) ? gx[q] : (q < DIM ? a.x_anc[q] : gx[DIM]);
        }
      } else if (pt < it.count) {
        v = ra.gh_x[(size_t)(it.start + pt) * D + q];
      }
      xin[k] = v;
    }
    __syncthreads();
    forward_tile<DIM, NCB, M_VALUE, ACT, RPW>(sh, a.subs[it.b].frag, bufH, ys, xin, L.S, tid, nthr, w, g, j, lane);
    float* tg = a.targets[it.a];
    for (int k = tid; k < it.count; k += nthr) {
      for (int o = 0; o < D; ++o) {
        float v = ys[o * NCOL + k];
        if (o == DIM && it.paired) v -= ys[o * NCOL + half + k];
        tg[(size_t)(it.start + k) * D + o] = v;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// evaluation post-processing (stitched field, master anchor pinning,
// per-snapshot pressure-mean removal, relative L2 errors)
// ---------------------------------------------------------------------------
__global__ void anchor_points_kernel(const float* x, int64_t n, int D, float a0, float a1, float a2, float* xa) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float an[3] = {a0, a1, a2};
  for (int q = 0; q < D - 1; ++q) xa[i * D + q] = an[q];
  xa[i * D + D - 1] = x[i * D + D - 1];   // the point's own time
}

// routed counts kept only for master subdomains (the anchor pass skips the rest)
__global__ void master_counts_kernel(const SubDev* subs, const int32_t* counts, int n_sub, int32_t* out) {
  for (int s = threadIdx.x; s < n_sub; s += blockDim.x) out[s] = subs[s].is_master ? counts[s] : 0;
}

__device__ __forceinline__ float block_sum256(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

// processed pressure of point i: p - p(x_anc, t) on master subdomains
__device__ __forceinline__ float eval_p(const EvalArgs& a, int64_t i) {
  const int D = a.D;
  float p = a.pred[i * D + D - 1];
  const int s = a.sub_id[i];
  if (s >= 0 && a.subs[s].is_master) p -= a.pa[i * D + D - 1];
  return p;
}

__global__ void eval_means_kernel(const EvalArgs a) {
  __shared__ float red[256];
  const int k = blockIdx.y;
  const int64_t b0 = a.snap_off[k], b1 = a.snap_off[k + 1];
  const int64_t lo = b0 + (int64_t)blockIdx.x * kEvalChunk;
  const int64_t hi = min(b1, lo + kEvalChunk);
  float sp = 0.f, sr = 0.f;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    sp += eval_p(a, i);
    sr += a.ref[i * a.D + a.D - 1];
  }
  sp = block_sum256(sp, red);
  sr = block_sum256(sr, red);
  if (threadIdx.x == 0) {
    a.mpart[((size_t)k * a.nblk + blockIdx.x) * 2 + 0] = sp;
    a.mpart[((size_t)k * a.nblk + blockIdx.x) * 2 + 1] = sr;
  }
}

__global__ void eval_err_kernel(const EvalArgs a) {
  __shared__ float red[256];
  const int k = blockIdx.y, D = a.D, dim = D - 1;
  const int64_t b0 = a.snap_off[k], b1 = a.snap_off[k + 1];
  float mp = 0.f, mr = 0.f;
  for (int b = 0; b < a.nblk; ++b) {
    mp += a.mpart[((size_t)k * a.nblk + b) * 2 + 0];
    mr += a.mpart[((size_t)k * a.nblk + b) * 2 + 1];
  }
  if (b1 > b0) {
    mp /= (float)(b1 - b0);
    mr /= (float)(b1 - b0);
  }
  const int64_t lo = b0 + (int64_t)blockIdx.x * kEvalChunk;
  const int64_t hi = min(b1, lo + kEvalChunk);
  float num[4] = {0.f, 0.f, 0.f, 0.f}, den[4] = {0.f, 0.f, 0.f, 0.f};
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    for (int q = 0; q < dim; ++q) {
      const float r = a.ref[i * D + q], e = a.pred[i * D + q] - r;
      num[q] += e * e;
      den[q] += r * r;
    }
    const float r = a.ref[i * D + dim] - mr;
    const float e = (eval_p(a, i) - mp) - r;
    num[dim] += e * e;
    den[dim] += r * r;
  }
  float* out = a.epart + ((size_t)k * a.nblk + blockIdx.x) * 2 * (D + 1);
  for (int q = 0; q < D; ++q) {
    const float vn = block_sum256(num[q], red);
    const float vd = block_sum256(den[q], red);
    if (threadIdx.x == 0) {
      out[2 * q] = vn;
      out[2 * q + 1] = vd;
    }
  }
}

// err[q] (velocity components), err[dim] (velocity vector), err[dim+1] (p)
__global__ void eval_final_kernel(const EvalArgs a) {
  if (threadIdx.x != 0) return;
  const int D = a.D, dim = D - 1;
  float num[4] = {0.f, 0.f, 0.f, 0.f}, den[4] = {0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < a.n_snap; ++k)
    for (int b = 0; b < a.nblk; ++b) {
      const float* e = a.epart + ((size_t)k * a.nblk + b) * 2 * (D + 1);
      for (int q = 0; q < D; ++q) {
        num[q] += e[2 * q];
        den[q] += e[2 * q + 1];
      }
    }
  float nv = 0.f, dv = 0.f;
  for (int q = 0; q < dim; ++q) {
    a.err_out[q] = sqrtf(num[q] / den[q]);
    nv += num[q];
    dv += den[q];
  }
  a.err_out[dim] = sqrtf(nv / dv);
  a.err_out[dim + 1] = sqrtf(num[dim] / den[dim]);
}

hipError_t launch_anchor_points(const float* x, int64_t n, int D, const float* x_anc, float* xa, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (nb)
    hipLaunchKernelGGL(anchor_points_kernel, dim3(nb), dim3(256), 0, s, x, n, D, x_anc[0], D > 2 ? x_anc[1] : 0.f,
                       D > 3 ? x_anc[2] : 0.f, xa);
  return hipGetLastError();
}

hipError_t launch_master_counts(const SubDev* subs, const int32_t* counts, int n_sub, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(master_counts_kernel, dim3(1), dim3(256), 0, s, subs, counts, n_sub, out);
  return hipGetLastError();
}

hipError_t launch_evaluate(const EvalArgs& a, hipStream_t s) {
  const dim3 grid(a.nblk, a.n_snap);
  hipLaunchKernelGGL(eval_means_kernel, grid, dim3(256), 0, s, a);
  hipLaunchKernelGGL(eval_err_kernel, grid, dim3(256), 0, s, a);
  hipLaunchKernelGGL(eval_final_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int step_value_points(int dim, int tile_points) {
  return 16 * (2 * dim + 2) * (tile_points / 16);
}

static int rows_per_wave(const Shape& sh) { return sh.NW > sh.NWV ? 2 : 1; }

int step_lds_floats(const Shape& sh, int tile_points) {
  const int NCB = (2 * sh.dim + 2) * (tile_points / 16);
  if (sh.split) return step_lds_split(sh.D, sh.Wp, sh.H, NCB, step_row_stride(sh.Wp)).total;
  return step_lds(sh.D, sh.Wp, sh.H, NCB, step_row_stride(sh.Wp)).total;
}

int query_lds_floats(const Shape& sh, int small) {
  return query_lds(sh.D, sh.Wp, small ? sh.dim + 1 : 2 * sh.dim + 2).total;
}

// Kernel instances: dimension, tile (16 or 32 collocation points), activation,
// row blocks per wave (2 above 8 row blocks; 16-point tiles only) and, for two
// row blocks, the column-split LDS plan.
template <int DIM, int PBP, int SS>
static const void* step_ptr_act(int act) {
  return act == ACT_SIN ? (const void*)step_kernel<DIM, PBP, ACT_SIN, 1, 0, SS>
                        : (const void*)step_kernel<DIM, PBP, ACT_TANH, 1, 0, SS>;
}
template <int DIM, int SS>
static const void* step_ptr_wide(int act, int split) {
  if (split) return act == ACT_SIN ? (const void*)step_kernel<DIM, 1, ACT_SIN, 2, 1, SS> : (const void*)step_kernel<DIM, 1, ACT_TANH, 2, 1, SS>;
  return act == ACT_SIN ? (const void*)step_kernel<DIM, 1, ACT_SIN, 2, 0, SS> : (const void*)step_kernel<DIM, 1, ACT_TANH, 2, 0, SS>;
}
template <int DIM>
static const void* step_ptr_dim(int tile_points, int act, int rpw, int split, int Wp) {
  if (rpw == 2) {
    switch (Wp) {
      case 160: return step_ptr_wide<DIM, 164>(act, split);
      case 208: return step_ptr_wide<DIM, 212>(act, split);
      default: return step_ptr_wide<DIM, 0>(act, split);
    }
  }
  if (tile_points == 32) return Wp <= 64 ? step_ptr_act<DIM, 2, 68>(act) : nullptr;
  switch (step_row_stride(Wp)) {
    case 68: return step_ptr_act<DIM, 1, 68>(act);
    case 100: return step_ptr_act<DIM, 1, 100>(act);
    default: return step_ptr_act<DIM, 1, 132>(act);
  }
}
static const void* step_ptr(int dim, int tile_points, int act, int rpw, int split, int Wp) {
  return dim == 2 ? step_ptr_dim<2>(tile_points, act, rpw, split, Wp) : step_ptr_dim<3>(tile_points, act, rpw, split, Wp);
}
const void* step_kernel_ptr(const Shape& sh, int tile_points) {
  if (rows_per_wave(sh) == 2 && tile_points != 16) return nullptr;
  return step_ptr(sh.dim, tile_points, sh.act, rows_per_wave(sh), sh.split, sh.Wp);
}
const void* prep_kernel_ptr() { return (const void*)prep_kernel; }
const void* slab_sum_kernel_ptr() { return (const void*)slab_sum_kernel; }
const void* grad_kernel_ptr() { return (const void*)grad_kernel; }
const void* clip_kernel_ptr() { return (const void*)clip_kernel; }
const void* adam_kernel_ptr() { return (const void*)adam_kernel; }

void grid_prep(const PrepArgs& a, dim3* grid, dim3* block) {
  *block = dim3(256);
  *grid = dim3((unsigned)((a.sh.frag_floats + 255) / 256), (unsigned)a.n_sub);
}
void grid_reduce(const ReduceArgs& a, dim3* grid, dim3* block) {
  *block = dim3(256);
  *grid = dim3((unsigned)((a.sh.P + 255) / 256), (unsigned)a.n_sub);
}
void grid_slab_sum(const ReduceArgs& a, dim3* grid, dim3* block) {
  *block = dim3(256);
  *grid = dim3((unsigned)((a.sh.slab_floats + 255) / 256), (unsigned)a.n_sub, (unsigned)a.n_chunks);
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t s) {
  dim3 grid, block;
  grid_prep(a, &grid, &block);
  hipLaunchKernelGGL(prep_kernel, grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, int tile_points, int n_wg, hipStream_t s) {
  const size_t lds = (size_t)a.lds_floats * sizeof(float);
  const void* k = step_kernel_ptr(a.sh, tile_points);
  if (!k) return hipErrorInvalidValue;
  const dim3 block(a.sh.NWV * 64);
  void* args[] = {const_cast<StepArgs*>(&a)};
  return hipLaunchKernel(k, dim3(n_wg), block, args, lds, s);
}

// Routed-query scratch held by the library, for callers that cannot
// allocate (pinn_query_noalloc).  Every GPU the library runs on holds its own
// copy for the life of the process.  Host code never passes this name to a
// kernel: the name is a host-side stand-in; the device address comes from
// noalloc_scratch_address, resolved once per device with that device current.
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

hipError_t noalloc_scratch_address(void** ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

// the same launch with events tied to the dispatch itself: e0 takes the
// kernel's start and e1 its end time stamp (either may be null)
hipError_t launch_step_timed(const StepArgs& a, int tile_points, int n_wg, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1) {
  const size_t lds = (size_t)a.lds_floats * sizeof(float);
  const void* k = step_kernel_ptr(a.sh, tile_points);
  if (!k) return hipErrorInvalidValue;
  const dim3 block(a.sh.NWV * 64);
  void* args[] = {const_cast<StepArgs*>(&a)};
  return hipExtLaunchKernel(k, dim3(n_wg), block, args, lds, s, e0, e1, 0);
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  dim3 grid, block;
  grid_slab_sum(a, &grid, &block);
  hipLaunchKernelGGL(slab_sum_kernel, grid, block, 0, s, a);
  grid_reduce(a, &grid, &block);
  hipLaunchKernelGGL(grad_kernel, grid, block, 0, s, a);
  if (a.clip > 0.f) hipLaunchKernelGGL(clip_kernel, dim3(a.n_sub), dim3(256), 0, s, a, (int)grid.x);
  hipLaunchKernelGGL(adam_kernel, grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_route(const RouteArgs& a, hipStream_t s) {
  if (a.n <= kRouteSmallMax) {
    hipLaunchKernelGGL(route_small_kernel, dim3(1), dim3(kRouteSmallThreads), 2 * sizeof(int) * (size_t)a.n_sub, s, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(route_zero_kernel, dim3(1), dim3(256), 0, s, a.counts, a.cursor, a.n_sub);
  const unsigned nb = (unsigned)((a.n + kRouteBlock - 1) / kRouteBlock);
  const size_t h = sizeof(int) * (size_t)a.n_sub;
  if (nb) hipLaunchKernelGGL(route_count_kernel, dim3(nb), dim3(kRouteBlock), h, s, a);
  hipLaunchKernelGGL(route_offsets_kernel, dim3(1), dim3(64), 0, s, a);
  if (nb) hipLaunchKernelGGL(route_scatter_kernel, dim3(nb), dim3(kRouteBlock), 2 * h, s, a);
  return hipGetLastError();
}

template <int DIM, int MODE, int RPW, int SMALL>
static const void* query_ptr_act(int act) {
  return act == ACT_SIN ? (const void*)query_kernel<DIM, MODE, ACT_SIN, RPW, SMALL>
                        : (const void*)query_kernel<DIM, MODE, ACT_TANH, RPW, SMALL>;
}
template <int DIM, int RPW>
static const void* query_ptr_mode(int mode, int act, int small) {
  if (mode == M_VALUE) return small ? query_ptr_act<DIM, M_VALUE, RPW, 1>(act) : query_ptr_act<DIM, M_VALUE, RPW, 0>(act);
  if (mode == M_GRAD) return small ? query_ptr_act<DIM, M_GRAD, RPW, 1>(act) : query_ptr_act<DIM, M_GRAD, RPW, 0>(act);
  return query_ptr_act<DIM, M_PDE, RPW, 0>(act);
}
static const void* query_ptr(int dim, int mode, int act, int rpw, int small) {
  if (dim == 2) return rpw == 2 ? query_ptr_mode<2, 2>(mode, act, small) : query_ptr_mode<2, 1>(mode, act, small);
  return rpw == 2 ? query_ptr_mode<3, 2>(mode, act, small) : query_ptr_mode<3, 1>(mode, act, small);
}
const void* query_kernel_ptr(const Shape& sh, int what, int small) {
  const int mode = (what == Q_VALUE) ? M_VALUE : (what == Q_UVPW ? M_GRAD : M_PDE);
  return query_ptr(sh.dim, mode, sh.act, rows_per_wave(sh), small);
}

static const void* exchange_ptr(int dim, int act, int rpw) {
  if (rpw == 2) {
    if (dim == 2) return act == ACT_SIN ? (const void*)exchange_kernel<2, ACT_SIN, 2> : (const void*)exchange_kernel<2, ACT_TANH, 2>;
    return act == ACT_SIN ? (const void*)exchange_kernel<3, ACT_SIN, 2> : (const void*)exchange_kernel<3, ACT_TANH, 2>;
  }
  if (dim == 2) return act == ACT_SIN ? (const void*)exchange_kernel<2, ACT_SIN, 1> : (const void*)exchange_kernel<2, ACT_TANH, 1>;
  return act == ACT_SIN ? (const void*)exchange_kernel<3, ACT_SIN, 1> : (const void*)exchange_kernel<3, ACT_TANH, 1>;
}
const void* exchange_kernel_ptr(const Shape& sh) { return exchange_ptr(sh.dim, sh.act, rows_per_wave(sh)); }

hipError_t launch_query(const QueryArgs& a, int n_wg, hipStream_t s) {
  if (n_wg >= 16) n_wg &= ~7;   // a multiple of the XCD count (see query_kernel)
  const size_t lds = (size_t)a.lds_floats * sizeof(float);
  const dim3 block(a.sh.NWV * 64);
  void* args[] = {const_cast<QueryArgs*>(&a)};
  return hipLaunchKernel(query_kernel_ptr(a.sh, a.what, a.small), dim3(n_wg), block, args, lds, s);
}

hipError_t launch_exchange(const ExchangeArgs& a, int n_wg, hipStream_t s) {
  const size_t lds = (size_t)a.lds_floats * sizeof(float);
  const dim3 block(a.sh.NWV * 64);
  void* args[] = {const_cast<ExchangeArgs*>(&a)};
  return hipLaunchKernel(exchange_kernel_ptr(a.sh), dim3(n_wg), block, args, lds, s);
}

// LDS above 64 KiB must be allowed per kernel before launch.
hipError_t set_lds_limits(int bytes) {
  hipError_t e = hipSuccess;
  auto allow = [&](const void* k) {
    const hipError_t r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (r != hipSuccess) e = r;
  };
  for (int dim = 2; dim <= 3; ++dim)
    for (int act = ACT_TANH; act <= ACT_SIN; ++act) {
      for (int wp : {64, 96, 128}) allow(step_ptr(dim, 16, act, 1, 0, wp));
      allow(step_ptr(dim, 32, act, 1, 0, 64));
      for (int wp : {160, 208, 256}) {   // the two constant strides and the argument
        allow(step_ptr(dim, 16, act, 2, 0, wp));
        allow(step_ptr(dim, 16, act, 2, 1, wp));
      }
      for (int rpw = 1; rpw <= 2; ++rpw) {
        for (int mode : {M_PDE, M_VALUE, M_GRAD}) {
          allow(query_ptr(dim, mode, act, rpw, 0));
          allow(query_ptr(dim, mode, act, rpw, 1));
        }
        allow(exchange_ptr(dim, act, rpw));
      }
    }
  return e;
}

}  // namespace ddp
