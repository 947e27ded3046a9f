// Adjoint of the cube (gradients through the pipeline: arXiv:2412.08265, Abstract and Sec. 1).
//
// Given G = dL/dC_raw, each in-field particle i of spaxel s needs four dot products over the
// telescope bins j of its spaxel's gradient row (Slin = bilinear SSP spectrum, linear in lambda):
//   s_m = sum_j G[s,j] Slin_i(q_ij)                        (mass, and the Jacobian term of v_los)
//   s_a = sum_j G[s,j] dSlin_i/dt_a(q_ij)                  (age direction of the bilinear cell)
//   s_z = sum_j G[s,j] dSlin_i/dt_z(q_ij)                  (metallicity direction)
//   Y   = sum_j G[s,j] lam_j dSlin_i/dq(q_ij)              (right-cell slope per node)
// from which the per-particle gradients follow in closed form (k_bwd_final). The directional
// derivatives are formed per bin from differences of the FP32 template values at each node
// (exact or nearly so) before they meet G, so no sum is a difference of nearly equal sums.
//
#include <type_traits>

#include "rubix_internal.h"

namespace rubix {

constexpr double kCkmsB = 299792.458;

hipError_t launch_prep_backward(const Table *dt, const TableHeader &h, int cap, hipStream_t s);

// Bin-edge table of the bin-mean jobs: edges 0 .. n_tel as the forward bin-mean kernel computes
// them (the node index split into integer part and fraction, and the edge wavelength).
__global__ __launch_bounds__(256) void k_bintab(const Table *__restrict__ T) {
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_BINTAB]; vb += gridDim.x) {
    const int jj = find_job(T, K_BINTAB, vb);
    const JobDev &J = jobs[jj];
    const int e = (int)((vb - J.vb_start[K_BINTAB]) * 256 + threadIdx.x);
    if (e > J.n_tel) continue;
    int qe;
    float fe, le;
    bin_edge(J, S, e, qe, fe, le);
    J.bintab[e] = make_float4(__int_as_float(qe), fe, le, 0.f);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One bin's terms of the four dots from the template values around its node: p_c at kk and q_c at
// kk + 1 in corner row c, interpolation fraction t, gradient weight g (0 where the bin is out of
// range) and the bin's Doppler factor lamf.
__device__ __forceinline__ void bwd_bin(float w0, float w1, float w2, float w3, float ta, float tz,
                                        float t, float g, float lamf, const float (&pv)[4],
                                        const float (&qv)[4], float &sm, float &sa, float &sz,
                                        float &y) {
  const float p0 = pv[0], q0 = qv[0], p1 = pv[1], q1 = qv[1];
  const float p2 = pv[2], q2 = qv[2], p3 = pv[3], q3 = qv[3];
  const float d0 = q0 - p0, d1 = q1 - p1, d2 = q2 - p2, d3 = q3 - p3;
  // S = sum_c w_c (p_c + t d_c) = P + t dS, with the slope sum dS needed for Y anyway
  const float dS = w0 * d0 + w1 * d1 + w2 * d2 + w3 * d3;
  const float S = fmaf(t, dS, w0 * p0 + w1 * p1 + w2 * p2 + w3 * p3);
  // age direction: (1-tz)(Tlin_2 - Tlin_0) + tz (Tlin_3 - Tlin_1); the difference of two corners'
  // linear interpolants is formed from the differences of their node values and of their slopes
  // (d_c = q_c - p_c), both taken before they meet G
  const float Aa = (1.f - tz) * fmaf(t, d2 - d0, p2 - p0) + tz * fmaf(t, d3 - d1, p3 - p1);
  // metallicity direction: (1-ta)(Tlin_1 - Tlin_0) + ta (Tlin_3 - Tlin_2)
  const float Az = (1.f - ta) * fmaf(t, d1 - d0, p1 - p0) + ta * fmaf(t, d3 - d2, p3 - p2);
  sm = fmaf(g, S, sm);
  sa = fmaf(g, Aa, sa);
  sz = fmaf(g, Az, sz);
  y = fmaf(g * lamf, dS, y);
}

__device__ __forceinline__ float4 ld_bintab(__amdgpu_buffer_rsrc_t rt, int j) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rt, j * 16, 0, 0));
}

__device__ __forceinline__ float ld_grad(__amdgpu_buffer_rsrc_t rg, int j) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, j * 4, 0, 0));
}

// One wave per particle, walking the telescope grid in windows of kCubeWaveBins bins (lane l takes
// bin jw + l; lanes 62 and 63 only stage, with the constants of the window's last bin, so their
// nodes stay in the window, and read no gradient). Each lane carries its bin's rest-frame node
// index at zero velocity in 40-bit fixed point and its wavelength in FP64 from window to window
// (one integer and one FP64 add per window instead of the split index's FP64 arithmetic).
// The windows whose 64 nodes n0 .. n0+63 (n0 = lane 0's node) lie inside the SSP grid form one
// contiguous run (n0 grows with the window's wavelength); for a particle whose span fits a
// window (the forward kernel's decision, carried in the record's sign) the run takes a loop of
// its own: the four corner rows are loaded with one coalesced load each (row base in scalar
// registers) and lane l stages, at node n0 + l, the cell's four bilinear basis rows (the first
// corner and three node-wise differences of corners) in the wave's LDS rows; each bin reads its
// two nodes of every basis row and accumulates, per basis row, the gradient-weighted
// interpolant and slope. The dots are linear in the rows, so the run's sums go back to the four
// dots once per particle. The windows before and after the run, and every window of a particle
// that does not fit, gather each lane's eight template values directly. Each lane accumulates its
// bins in increasing order; the wave's sums are reduced in FP64.
__global__ __launch_bounds__(256) void k_bwd_dots(const Table *__restrict__ T) {
  __shared__ float rows[4][4][64];     // [wave][basis row U0..U3][node - n0]
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  const float *__restrict__ flux = S.flux;
  const int nl = S.n_lam;
  const int o1 = nl, o2 = S.n_met * nl, o3 = o2 + nl;
  // the wave index is wave-uniform: say so, so that per-particle values live in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const uint32_t fbytes = (uint32_t)S.n_age * (uint32_t)S.n_met * (uint32_t)nl * 4u;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)flux, (short)0, (int)fbytes, 0x00020000);
  // byte offsets of this lane's node in the four corner rows relative to corner (ja, jz)
  uint32_t lo[4] = {(uint32_t)lane * 4u, (uint32_t)(lane + o1) * 4u, (uint32_t)(lane + o2) * 4u,
                    (uint32_t)(lane + o3) * 4u};
  const uint32_t oc[4] = {0u, (uint32_t)o1 * 4u, (uint32_t)o2 * 4u, (uint32_t)o3 * 4u};
  const int jl = min(lane, kCubeWaveBins - 1);
  // gradient offsets: lanes 62 and 63 point past any row, so their loads return 0
  const uint32_t gofs = lane < kCubeWaveBins ? (uint32_t)lane * 4u : 0x40000000u;
  float *wr = &rows[w][0][0];
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_BWD]; vb += gridDim.x) {
    const int jj = find_job(T, K_BWD, vb);
    const JobDev &J = jobs[jj];
    const int64_t pbase = (vb - J.vb_start[K_BWD]) * kBwdParticles;
    const int n_in = J.seg_off[J.n_s];
    const int64_t step_x = (int64_t)kCubeWaveBins * J.qrx;
    const double step_l = (double)kCubeWaveBins * J.tel_step;
    for (int q = w; q < kBwdParticles; q += 4) {
      const int64_t p = pbase + q;
      if (p >= n_in) break;
      const PrepRec r = J.prep[p];
      // the record is the wave's (a vector load of one address): its integers in scalar registers
      const int spx = __builtin_amdgcn_readfirstlane(r.spaxel);
      const int rrow = __builtin_amdgcn_readfirstlane(r.row);
      const int jo = __builtin_amdgcn_readfirstlane(r.pad);     // input index: where the dots go
      const float w0 = r.a[0], w1 = r.a[1], w2 = r.a[2], w3 = r.a[3];
      const float ta = w2 + w3, tz = w1 + w3;   // bilinear fractions recovered from the weights
      const bool fits = rrow >= 0;
      const int row = prep_row(rrow);
      // the particle's gradient row: loads past its last bin return 0
      const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(J.grad_raw + (int64_t)spx * J.n_tel), (short)0, J.n_tel * 4, 0x00020000);
      const float g = r.g;
      const bool loglam = __builtin_amdgcn_readfirstlane(J.log_lambda) != 0;
      float sm = 0.f, sa = 0.f, sz = 0.f, y = 0.f;
      // this lane's bin (jw + jl) in the current window: fixed-point rest index and wavelength
      int64_t Qx = J.q0x + (int64_t)jl * J.qrx;
      double lamd = J.tel_start + (double)jl * J.tel_step;
      int jw = 0;
      // node index of this lane's bin in window jw, the window's lowest node n0 (lane 0's) and
      // the lane's gradient value
      auto locate = [&](float &lamf, float &tau, int &k, int &n0, float &gj) {
        const int qi = (int)(Qx >> 40);
        const float qf = (float)(uint32_t)((uint64_t)Qx >> 8) * 0x1p-32f;
        lamf = loglam ? 1.0f : (float)lamd;
        const float tq = fmaf(-lamf, g, qf);
        const float fl = floorf(tq);
        tau = tq - fl;
        k = qi + (int)fminf(fmaxf(fl, -1.0e8f), 1.0e8f);
        n0 = __builtin_amdgcn_readfirstlane(k);
        gj = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                           rg, gofs + (uint32_t)jw * 4u, 0, 0));
      };
      // direct gathers: bins whose node lies outside the SSP grid carry no gradient (a select,
      // not a store under a branch); the last node takes the last interval with t = 1
      auto general = [&](float lamf, float tau, int k, float gj) {
        const bool ok = (k >= 0) & ((k < nl - 1) | ((k == nl - 1) & (tau == 0.f)));
        const float g = ok ? gj : 0.f;
        const int kk = min(max(k, 0), nl - 2);
        const float t = (k > kk) ? 1.f : tau;
        const uint32_t bo = (uint32_t)(row + kk) * 4u;
        float pv[4], qv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          pv[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, bo + oc[c], 0, 0));
          qv[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, bo + oc[c] + 4u, 0, 0));
        }
        bwd_bin(w0, w1, w2, w3, ta, tz, t, g, lamf, pv, qv, sm, sa, sz, y);
      };
      if (fits) {
        // windows before the run
        for (; jw < J.n_tel; jw += kCubeWaveBins, Qx += step_x, lamd += step_l) {
          float lamf, tau, gj;
          int k, n0;
          locate(lamf, tau, k, n0, gj);
          if (n0 >= 0 && n0 + 63 <= nl - 1) break;
          general(lamf, tau, k, gj);
        }
        // the run: every lane's node k lies in [n0, n0 + 62], inside [0, n - 2]. The four dots
        // are linear in the template rows, so the run accumulates them per row of the cell's
        // bilinear basis U0 = T0, U1 = T1 - T0 (metallicity), U2 = T2 - T0 (age),
        // U3 = T3 - T2 - T1 + T0 (cross): S = U0 + tz U1 + ta U2 + ta tz U3, the age direction
        // (1-tz)(T2-T0) + tz(T3-T1) = U2 + tz U3, the metallicity direction U1 + ta U3. Per
        // basis row b the lane sums e_b = sum G (U_b(k) + tau dU_b) and f_b = sum G lam dU_b,
        // dU_b = U_b(k+1) - U_b(k); the node differences are taken on FP32 node values before
        // any sum (on fine grids the spectrum changes by 1e-3 of itself per node).
        // One copy of the loop per grid kind (log grids: the Doppler factor of g is 1). Within the
        // run a particle's node indices stay far inside the int range (its span fits a window,
        // which bounds |lam g| by lam / dlam_tel), so the index is one floor-and-convert.
        float e0 = 0.f, e1 = 0.f, e2 = 0.f, e3 = 0.f, f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
        auto run = [&](auto log_grid) {
          for (; jw < J.n_tel; jw += kCubeWaveBins, Qx += step_x, lamd += step_l) {
            // the lane offsets pass through an empty asm each iteration, so their widening to
            // 64 bits stays next to the loads and the loads take the scalar-base form
            asm volatile("" : "+v"(lo[0]), "+v"(lo[1]), "+v"(lo[2]), "+v"(lo[3]));
            const int qi = (int)(Qx >> 40);
            const float qf = (float)(uint32_t)((uint64_t)Qx >> 8) * 0x1p-32f;
            const float lamf = decltype(log_grid)::value ? 1.0f : (float)lamd;
            const float tq = fmaf(-lamf, g, qf);
            const int k = qi + floor_i32(tq);
            const int n0 = __builtin_amdgcn_readfirstlane(k);
            if (!(n0 >= 0 && n0 + 63 <= nl - 1)) break;
            const float tau = __builtin_amdgcn_fractf(tq);
            // the gradient of the lane's bin: the window's offset goes into the lane's offset,
            // which the buffer's range check covers (bins past the row's end read 0)
            const float gj = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(rg, gofs + (uint32_t)jw * 4u, 0, 0));
            const GChar *wb = (const GChar *)flux + (uint32_t)(row + n0) * 4u;
            float st[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) st[c] = *(const GFloat *)(wb + lo[c]);
            const float u1 = st[1] - st[0];
            wr[lane] = st[0];
            wr[64 + lane] = u1;
            wr[128 + lane] = st[2] - st[0];
            wr[192 + lane] = (st[3] - st[2]) - u1;
            __builtin_amdgcn_wave_barrier();
            const int i = k - n0;
            float b0[4], b1[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              b0[b] = wr[64 * b + i];
              b1[b] = wr[64 * b + i + 1];
            }
            __builtin_amdgcn_wave_barrier();
            const float gl = gj * lamf;
            float du[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) du[b] = b1[b] - b0[b];
            e0 = fmaf(gj, fmaf(tau, du[0], b0[0]), e0);
            e1 = fmaf(gj, fmaf(tau, du[1], b0[1]), e1);
            e2 = fmaf(gj, fmaf(tau, du[2], b0[2]), e2);
            e3 = fmaf(gj, fmaf(tau, du[3], b0[3]), e3);
            f0 = fmaf(gl, du[0], f0);
            f1 = fmaf(gl, du[1], f1);
            f2 = fmaf(gl, du[2], f2);
            f3 = fmaf(gl, du[3], f3);
          }
        };
        if (loglam) run(std::true_type{});
        else run(std::false_type{});
        // back to the four dots (the bilinear fractions from the record's weights)
        const float tt = ta * tz;
        sm += fmaf(tt, e3, fmaf(ta, e2, fmaf(tz, e1, e0)));
        sa += fmaf(tz, e3, e2);
        sz += fmaf(ta, e3, e1);
        y += fmaf(tt, f3, fmaf(ta, f2, fmaf(tz, f1, f0)));
      }
      // windows after the run, or every window of a particle that does not fit
      for (; jw < J.n_tel; jw += kCubeWaveBins, Qx += step_x, lamd += step_l) {
        float lamf, tau, gj;
        int k, n0;
        locate(lamf, tau, k, n0, gj);
        general(lamf, tau, k, gj);
      }
      const double Sm = wave_sum(sm), Sa = wave_sum(sa), Sz = wave_sum(sz), Y = wave_sum(y);
      if (lane == 0) {
        double *d = J.dots + (int64_t)jo * 4;
        d[0] = Sm; d[1] = Sa; d[2] = Sz; d[3] = Y;
      }
    }
  }
}

// Bin-mean jobs. A bin's value is the integral of the particle's linear interpolants over the
// bin's rest-frame node interval [q_lo, q_hi] clipped to [0, n-1], so the dots become
//   s_m, s_a, s_z = sum_j G[s,j] x (integral over bin j of Slin, of its age direction, of its
//                   metallicity direction),
//   Y = sum_j G[s,j] (lam_hi Slin(q_hi) [q_hi inside] - lam_lo Slin(q_lo) [q_lo inside]),
// Y holding the Leibniz terms of the moving limits (an edge clipped to the grid's end does not
// move, so it contributes nothing; "inside" is 0 < q < n-1). Where both edges are inside,
// lam_hi S_hi - lam_lo S_lo is formed as lam_lo (S_hi - S_lo) + dlam S_hi, with S_hi - S_lo
// summed from the segments' slopes, so a bin's term is not a difference of two nearly equal
// products.

// Terms of one node segment [x, xe] (fractions) between node values p_c and q_c of the corner
// rows: the integrals of Slin and of its two directions, and Slin's slope dS (per node).
struct SegTerms {
  float is, ia, iz, ds, p;
};
__device__ __forceinline__ SegTerms seg_terms(float w0, float w1, float w2, float w3, float ta,
                                              float tz, const float (&pv)[4], const float (&qv)[4],
                                              float x, float xe) {
  SegTerms o;
  o.p = w0 * pv[0] + w1 * pv[1] + w2 * pv[2] + w3 * pv[3];
  o.ds = w0 * (qv[0] - pv[0]) + w1 * (qv[1] - pv[1]) + w2 * (qv[2] - pv[2]) + w3 * (qv[3] - pv[3]);
  // age and metallicity directions at the two nodes, differences taken before the sums
  const float ap = (1.f - tz) * (pv[2] - pv[0]) + tz * (pv[3] - pv[1]);
  const float aq = (1.f - tz) * (qv[2] - qv[0]) + tz * (qv[3] - qv[1]);
  const float zp = (1.f - ta) * (pv[1] - pv[0]) + ta * (pv[3] - pv[2]);
  const float zq = (1.f - ta) * (qv[1] - qv[0]) + ta * (qv[3] - qv[2]);
  o.is = seg_integral(o.p, o.p + o.ds, x, xe);
  o.ia = seg_integral(ap, aq, x, xe);
  o.iz = seg_integral(zp, zq, x, xe);
  return o;
}

// One wave per particle, walking the telescope grid in windows of kBinWaveBins bins (lane l takes
// bin jw + l and splits its lower edge; the upper edge is the next lane's; the last lanes only
// stage). Where every bin of the window spans at most two node segments and the window's bins
// span at most 63 nodes, the four corner rows at nodes n0 .. n0+63 (n0 = lane 0's lower node)
// are staged in the wave's LDS rows with one coalesced load each; each lane reads the two nodes
// of its edge's segment and integrates that segment, and a bin combines its two edges' partial
// integrals. Otherwise each lane walks its bin's segments with direct gathers. Each lane
// accumulates its bins in increasing order; the wave's sums are reduced in FP64.
// Log grids (kLog): the integrals run over rest wavelength (each segment's partials carry the
// weights E1 and Phi and the node's wavelength, as in the forward kernel), each bin's gradient
// is divided by the bin's width, and the Leibniz term of an edge is Slin lam_edge dln (both
// edges move by dq/dbeta = -1/((1+beta) dln)); where both edges are inside,
// lam_hi S_hi - lam_lo S_lo = lam_lo ((S_hi - S_lo) + S_hi expm1(dln_tel)), the rest-frame
// edges' wavelength ratio being e^{dln_tel}.
template <bool kLog>
__device__ __forceinline__ void bwd_dots_bin(const Table *__restrict__ T) {
  __shared__ float rows[4][4][64];     // [wave][corner][node - n0]
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  const int nl = S.n_lam;
  const int o1 = nl, o2 = S.n_met * nl, o3 = o2 + nl;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const uint32_t fbytes = (uint32_t)S.n_age * (uint32_t)S.n_met * (uint32_t)nl * 4u;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)S.flux, (short)0, (int)fbytes, 0x00020000);
  const uint32_t lb[4] = {(uint32_t)lane * 4u, (uint32_t)(lane + o1) * 4u,
                          (uint32_t)(lane + o2) * 4u, (uint32_t)(lane + o3) * 4u};
  const uint32_t oc[4] = {0u, (uint32_t)o1 * 4u, (uint32_t)o2 * 4u, (uint32_t)o3 * 4u};
  float *wr = &rows[w][0][0];
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_BWDB]; vb += gridDim.x) {
    const int jj = find_job(T, K_BWDB, vb);
    const JobDev &J = jobs[jj];
    const int64_t pbase = (vb - J.vb_start[K_BWDB]) * kBwdParticles;
    const int n_in = J.seg_off[J.n_s];
    const float dlam = (float)J.tel_step;
    // log grids: node wavelengths, whole-segment weights, the edges' wavelength ratio - 1, and
    // the bins' widths lam_j 2 sinh(dln_tel / 2) = w0 e^{j dln_tel}
    const float lam0 = (float)S.lam_start, dln = (float)S.lam_step;
    const float e1h = expm1_small(dln), phh = phi_small(dln);
    const float rt1 = kLog ? (float)expm1(J.tel_step) : 0.f;
    const float inv_w0 = kLog ? (float)(1.0 / (J.tel_start * 2.0 * sinh(0.5 * J.tel_step))) : 0.f;
    const __amdgpu_buffer_rsrc_t rt =
        __builtin_amdgcn_make_buffer_rsrc((void *)J.bintab, (short)0, (J.n_tel + 1) * 16, 0x00020000);
    for (int q = w; q < kBwdParticles; q += 4) {
      const int64_t p = pbase + q;
      if (p >= n_in) break;
      const PrepRec r = J.prep[p];
      const int spx = __builtin_amdgcn_readfirstlane(r.spaxel);
      const int row = prep_row(__builtin_amdgcn_readfirstlane(r.row));
      const int jo = __builtin_amdgcn_readfirstlane(r.pad);
      const float *__restrict__ G = J.grad_raw + (int64_t)spx * J.n_tel;
      const __amdgpu_buffer_rsrc_t rg =
          __builtin_amdgcn_make_buffer_rsrc((void *)G, (short)0, J.n_tel * 4, 0x00020000);
      const float w0 = r.a[0], w1 = r.a[1], w2 = r.a[2], w3 = r.a[3];
      const float ta = w2 + w3, tz = w1 + w3;
      float sm = 0.f, sa = 0.f, sz = 0.f, y = 0.f;
      for (int jw = 0; jw < J.n_tel; jw += kBinWaveBins) {
        const bool act = (lane < kBinWaveBins) && (jw + lane < J.n_tel);
        const int jc = min(jw + min(lane, kBinWaveBins - 1), J.n_tel - 1);
        float graw = ld_grad(rg, jc);
        if (kLog) graw *= inv_w0 * expf(-(float)jc * dlam);      // / the bin's width
        // lane l splits edge jw + l, the lower edge of its bin; the upper edge is the next lane's
        // (lanes past the window's last edge take it, so the node span stays the bins')
        const float4 lo = ld_bintab(rt, min(jw + min(lane, kBinWaveBins), J.n_tel));
        const float tl = fmaf(-lo.z, r.g, lo.y);
        int klo = __float_as_int(lo.x) + floor_i32(tl);
        float a = __builtin_amdgcn_fractf(tl);
        const bool in_lo = (klo > 0 || (klo == 0 && a > 0.f)) && klo < nl - 1;
        clip_node(klo, a, nl);
        const int khi = __shfl_down(klo, 1, 64);
        const float b = __shfl_down(a, 1, 64);
        const bool in_hi = __shfl_down((int)in_lo, 1, 64) != 0;
        const float lhi = __shfl_down(lo.z, 1, 64);
        // empty: both edges clipped to the same point of the grid
        const bool empty = klo > khi || (klo == khi && !(a < b));
        const int n0 = __builtin_amdgcn_readfirstlane(klo);
        const int nmax = __builtin_amdgcn_readlane(khi, 63) + 1;
        const bool multi = !empty && (khi - klo > 1);
        float Is = 0.f, Ia = 0.f, Iz = 0.f, D = 0.f, s_lo = 0.f, s_hi = 0.f;
        // log grids: wavelength of the lower edge's node and of the edge itself (every lane, so
        // that the previous lane can take its upper edge's)
        float lamk_lo = 0.f, lam_lo = 0.f;
        if (kLog) {
          lamk_lo = lam0 * expf((float)klo * dln);
          lam_lo = fmaf(lamk_lo, expm1_small(a * dln), lamk_lo);
        }
        if (nmax - n0 <= 63 && !__builtin_amdgcn_ballot_w64(multi)) {
          // every lane's nodes klo .. khi+1 lie in n0 .. n0+63; rows read past the end of a row
          // (or of the grid, as zeros) only feed lanes that do not use them
          const uint32_t so = (uint32_t)(row + n0) * 4u;
          float st[4];
#pragma unroll
          for (int c = 0; c < 4; ++c)
            st[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lb[c] + so, 0, 0));
#pragma unroll
          for (int c = 0; c < 4; ++c) wr[c * 64 + lane] = st[c];
          __builtin_amdgcn_wave_barrier();
          const int i = min(max(klo - n0, 0), 62);
          float pv[4], qv[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            pv[c] = wr[c * 64 + i];
            qv[c] = wr[c * 64 + i + 1];
          }
          __builtin_amdgcn_wave_barrier();
          // each lane integrates its own edge's segment, from the node to the edge (P) and whole
          // (T); a bin's integrals are P(upper edge) - P(lower edge), plus the lower segment's T
          // when the upper edge lies in the next segment, the upper values coming from the next
          // lane
          SegTerms te = seg_terms(w0, w1, w2, w3, ta, tz, pv, qv, 0.f, a);
          const float ap = (1.f - tz) * (pv[2] - pv[0]) + tz * (pv[3] - pv[1]);
          const float aq = (1.f - tz) * (qv[2] - qv[0]) + tz * (qv[3] - qv[1]);
          const float zp = (1.f - ta) * (pv[1] - pv[0]) + ta * (pv[3] - pv[2]);
          const float zq = (1.f - ta) * (qv[1] - qv[0]) + ta * (qv[3] - qv[2]);
          float TS = fmaf(0.5f, te.ds, te.p), TA = 0.5f * (ap + aq), TZ = 0.5f * (zp + zq);
          if (kLog) {
            // the same partials and wholes over rest wavelength
            const float lamk = lamk_lo;
            te.is = log_partial(lamk, te.p, te.ds, a, dln);
            te.ia = log_partial(lamk, ap, aq - ap, a, dln);
            te.iz = log_partial(lamk, zp, zq - zp, a, dln);
            TS = lamk * fmaf(te.p, e1h, te.ds * phh);
            TA = lamk * fmaf(ap, e1h, (aq - ap) * phh);
            TZ = lamk * fmaf(zp, e1h, (zq - zp) * phh);
          }
          const float Se = fmaf(a, te.ds, te.p);
          const float PSn = __shfl_down(te.is, 1, 64), PAn = __shfl_down(te.ia, 1, 64);
          const float PZn = __shfl_down(te.iz, 1, 64), dSn = __shfl_down(te.ds, 1, 64);
          const float Sn = __shfl_down(Se, 1, 64);
          const bool two = khi > klo;
          Is = (PSn - te.is) + (two ? TS : 0.f);
          Ia = (PAn - te.ia) + (two ? TA : 0.f);
          Iz = (PZn - te.iz) + (two ? TZ : 0.f);
          D = two ? fmaf(dSn, b, te.ds * (1.f - a)) : te.ds * (b - a);
          s_lo = Se;
          s_hi = Sn;
        } else if (!empty) {
          // any number of segments, gathered from the template grid
          for (int k = klo; k <= khi; ++k) {
            const uint32_t e = (uint32_t)(row + k) * 4u;
            float pv[4], qv[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              pv[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, e + oc[c], 0, 0));
              qv[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, e + oc[c] + 4u, 0, 0));
            }
            const float x = k == klo ? a : 0.f, xe = k == khi ? b : 1.f;
            const SegTerms t = seg_terms(w0, w1, w2, w3, ta, tz, pv, qv, x, xe);
            if (kLog) {
              const float lamk = lam0 * expf((float)k * dln);
              const float ap = (1.f - tz) * (pv[2] - pv[0]) + tz * (pv[3] - pv[1]);
              const float aq = (1.f - tz) * (qv[2] - qv[0]) + tz * (qv[3] - qv[1]);
              const float zp = (1.f - ta) * (pv[1] - pv[0]) + ta * (pv[3] - pv[2]);
              const float zq = (1.f - ta) * (qv[1] - qv[0]) + ta * (qv[3] - qv[2]);
              Is += log_partial(lamk, t.p, t.ds, xe, dln) - log_partial(lamk, t.p, t.ds, x, dln);
              Ia += log_partial(lamk, ap, aq - ap, xe, dln) - log_partial(lamk, ap, aq - ap, x, dln);
              Iz += log_partial(lamk, zp, zq - zp, xe, dln) - log_partial(lamk, zp, zq - zp, x, dln);
            } else {
              Is += t.is;
              Ia += t.ia;
              Iz += t.iz;
            }
            D = fmaf(t.ds, xe - x, D);
            s_lo = k == klo ? fmaf(a, t.ds, t.p) : s_lo;
            s_hi = k == khi ? fmaf(b, t.ds, t.p) : s_hi;
          }
        }
        float e;
        if (kLog) {
          // Leibniz terms per unit of dq/dbeta: Slin lam dln at each edge
          const float lam_hi = __shfl_down(lam_lo, 1, 64);
          if (in_lo && in_hi) e = dln * lam_lo * fmaf(s_hi, rt1, D);
          else e = dln * ((in_hi ? lam_hi * s_hi : 0.f) - (in_lo ? lam_lo * s_lo : 0.f));
        } else if (in_lo && in_hi) {
          e = fmaf(lo.z, D, dlam * s_hi);
        } else {
          e = (in_hi ? lhi * s_hi : 0.f) - (in_lo ? lo.z * s_lo : 0.f);
        }
        // an empty bin, or a lane past the window's bins, adds nothing
        const float g = (act && !empty) ? graw : 0.f;
        sm = fmaf(g, Is, sm);
        sa = fmaf(g, Ia, sa);
        sz = fmaf(g, Iz, sz);
        y = fmaf(g, e, y);
      }
      const double Sm = wave_sum(sm), Sa = wave_sum(sa), Sz = wave_sum(sz), Y = wave_sum(y);
      if (lane == 0) {
        double *d = J.dots + (int64_t)jo * 4;
        d[0] = Sm; d[1] = Sa; d[2] = Sz; d[3] = Y;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_bwd_dots_bin(const Table *__restrict__ T) {
  bwd_dots_bin<false>(T);
}

// The log instance holds more live values (the weights of three directions). Its register budget
// is set for 8 waves per SIMD: a few values spill, and it runs at 163 ms on the 1e7 galaxy against
// 210 ms at the 4 waves its natural 114 registers allow.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_bwd_dots_bin_log(
    const Table *__restrict__ T) {
  bwd_dots_bin<true>(T);
}

__device__ __forceinline__ int cell_of_b(const double *thr, int n, double x) {
  if (!(x > thr[0])) return 0;
  if (x >= thr[n - 1]) return n - 2;
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (thr[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kFinThreads) void k_bwd_final(const Table *__restrict__ T) {
  __shared__ double red[3][kFinThreads];
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  const int t = threadIdx.x;
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_FIN]; vb += gridDim.x) {
    const int jj = find_job(T, K_FIN, vb);
    const JobDev &J = jobs[jj];
    const int64_t blk = vb - J.vb_start[K_FIN];
    // in input order: the particle arrays, its dots and its gradients are read and written
    // coalesced; particles outside the field (key n_s) get zeros
    const int64_t i = blk * kFinThreads + t;
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    if (i < J.n) {
      const int64_t j = i;
      float gm = 0.f, ga = 0.f, gz = 0.f, gv = 0.f;
      // a particle whose line-of-sight velocity is not finite adds nothing to the cube (its
      // forward weights are zero), so it carries no gradient and no angle term either
      if (J.key[j] < J.n_s && isfinite(J.vlos[j])) {
        const double age = J.age[j], m = J.mass[j], met = J.met[j], v = J.vlos[j];
        const int na = S.n_age, nz = S.n_met;
        const bool in_a = (age >= S.age_thr[0]) && (age <= S.age_thr[na - 1]);
        const bool in_z = (met >= S.met[0]) && (met <= S.met[nz - 1]);
        const int ja = cell_of_b(S.age_thr, na, age);
        const int jz = cell_of_b(S.met, nz, met);
        const double *X = J.dots + j * 4;
        const double sm = X[0], sa = X[1], sz = X[2], Y = X[3];
        const double beta = v / kCkmsB;
        const double opz = 1.0 + J.z_sys;
        // bin-centre sampling: the Jacobian 1/((1+z)(1+beta)) scales the sample and moves with
        // beta; the bin mean carries the constant dlam_ssp/dlam_tel instead
        const double jac = J.resample ? J.bin_scale : 1.0 / (opz * (1.0 + beta));
        const double fs = J.flux_scale;
        const double A = fs * m * jac;
        gm = (float)(fs * jac * sm);
        if (in_a) ga = (float)(A * sa / (S.log_age[ja + 1] - S.log_age[ja]) / (age * 2.302585092994046));
        if (in_z) gz = (float)(A * sz / (S.met[jz + 1] - S.met[jz]));
        const double dJ = J.resample ? 0.0 : -jac / (1.0 + beta);
        // dq/dbeta per unit of the bin factor accumulated in Y (lambda on linear grids, 1 on
        // log grids, where q = Q - ln(1+beta)/dln; the edge wavelength for the bin mean)
        const double dq = J.log_lambda ? -1.0 / ((1.0 + beta) * S.lam_step)
                                       : -1.0 / (opz * (1.0 + beta) * (1.0 + beta) * S.lam_step);
        const double dbeta = fs * m * (dJ * sm + jac * dq * Y);
        const double dv = dbeta / kCkmsB;
        gv = (float)dv;
        const double vx = J.vx[j], vy = J.vy[j], vz = J.vz[j];
        c0 = dv * (J.dR2[0] * vx + J.dR2[1] * vy + J.dR2[2] * vz);
        c1 = dv * (J.dR2[3] * vx + J.dR2[4] * vy + J.dR2[5] * vz);
        c2 = dv * (J.dR2[6] * vx + J.dR2[7] * vy + J.dR2[8] * vz);
      }
      J.d_mass[j] = gm;
      J.d_age[j] = ga;
      J.d_met[j] = gz;
      J.d_vlos[j] = gv;
      if (J.d_vel) {
        J.d_vel[j] = (float)((double)gv * J.R[6]);
        J.d_vel[(int64_t)J.n + j] = (float)((double)gv * J.R[7]);
        J.d_vel[2 * (int64_t)J.n + j] = (float)((double)gv * J.R[8]);
      }
    }
    red[0][t] = c0; red[1][t] = c1; red[2][t] = c2;
    __syncthreads();
    for (int off = kFinThreads / 2; off > 0; off >>= 1) {
      if (t < off) {
        red[0][t] += red[0][t + off];
        red[1][t] += red[1][t + off];
        red[2][t] += red[2][t + off];
      }
      __syncthreads();
    }
    if (t < 3) J.ang_part[blk * 3 + t] = red[t][0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_bwd_angles(const Table *__restrict__ T) {
  __shared__ double red[3][256];
  const JobDev *jobs = table_jobs(T);
  const int t = threadIdx.x;
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_ANG]; vb += gridDim.x) {
    const int jj = find_job(T, K_ANG, vb);
    const JobDev &J = jobs[jj];
    const int nb = J.n_fin_blocks;
    const int per = (nb + 255) / 256;
    const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int b = b0; b < b1; ++b) {
      a0 += J.ang_part[b * 3 + 0];
      a1 += J.ang_part[b * 3 + 1];
      a2 += J.ang_part[b * 3 + 2];
    }
    red[0][t] = a0; red[1][t] = a1; red[2][t] = a2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (t < off) {
        red[0][t] += red[0][t + off];
        red[1][t] += red[1][t + off];
        red[2][t] += red[2][t + off];
      }
      __syncthreads();
    }
    if (t < 3) J.d_angles[t] = red[t][0];
    __syncthreads();
  }
}

static inline int grid_for(int64_t total, int cap) {
  if (total <= 0) return 0;
  int64_t g = total;
  if (cap > 0 && g > cap) g = cap;
  if (g > 0x7fffffff) g = 0x7fffffff;
  return (int)g;
}

hipError_t launch_backward(const Table *dt, const TableHeader &h, int cap, hipStream_t s) {
  hipError_t e = launch_prep_backward(dt, h, cap, s);
  if (e != hipSuccess) return e;
  int g;
  if ((g = grid_for(h.total[K_BINTAB], cap))) hipLaunchKernelGGL(k_bintab, dim3(g), dim3(256), 0, s, dt);
  if ((g = grid_for(h.total[K_BWD], cap))) hipLaunchKernelGGL(k_bwd_dots, dim3(g), dim3(256), 0, s, dt);
  if ((g = grid_for(h.total[K_BWDB], cap))) {
    if (h.ssp.log_lambda)
      hipLaunchKernelGGL(k_bwd_dots_bin_log, dim3(g), dim3(256), 0, s, dt);
    else
      hipLaunchKernelGGL(k_bwd_dots_bin, dim3(g), dim3(256), 0, s, dt);
  }
  if ((g = grid_for(h.total[K_FIN], cap))) hipLaunchKernelGGL(k_bwd_final, dim3(g), dim3(kFinThreads), 0, s, dt);
  if ((g = grid_for(h.total[K_ANG], cap))) hipLaunchKernelGGL(k_bwd_angles, dim3(g), dim3(256), 0, s, dt);
  return hipGetLastError();
}

}  // namespace rubix
