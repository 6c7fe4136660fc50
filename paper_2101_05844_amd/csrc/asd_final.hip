// FP64 per-neuron sums and backward pass of the final bound of an FP32 plan
// in sign classes, for one count of active masks: compiled once per count
// with -DASD_NM=<count>.
//
// For neuron o of ReLU layer k the final bound needs, over its active masks
// q with multipliers b_q (eq:dual-active-set),
//   r1 = sum_q b_q LI_q[o] and r0 = sum_q b_q (LI_q[o] + UI_q[o]),
// where LI_q sums W Lcheck over the taps j in mask q and UI_q sums W Ucheck
// over the others.  Exchanging the sums: r1 = sum_j wl_j PD_j and
// r0 = r1 + sum_j wu_j (B - PD_j), with wl, wu the tap's W Lcheck, W Ucheck,
// B = sum_q b_q and PD_j = sum over the masks containing j of b_q.  With
// P = sum over z_q[o] = 1 of b_q, Q_q = (1 - z_q[o]) b_q and X = sum_q
// xbit_q[j] Q_q (no point box at j), PD_j = B - X for w > 0, P + X for w < 0,
// B on a point box (a zero weight contributes nothing).  One walk over the
// fan-in serves every mask; the weight is uniform across a wave, so its
// sign class is a uniform branch.
#include "asd_adjoint.h"
#include "asd_plan.h"

#ifndef ASD_NM
#error "compile with -DASD_NM=<active mask count>"
#endif

namespace asd {

namespace {

// NW waves split the fan-in; DV: a dense layer over channels of 4k positions
// whose fan-in splits into multiples of 4 taps (one vector load per 4 taps).
template <int NM, int NW, bool DV>
__global__ void __launch_bounds__(kWave * NW) k_final_sums_sc(MaskArgs<float> A, const GwIn<float>* rec) {
    static_assert(NW >= CB, "one wave per channel finishes the sums");
    extern __shared__ unsigned char red_raw[];
    double* red = reinterpret_cast<double*>(red_raw);  // [NW][CB][2][64]
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S;
    const bool colok = col < g.out.cols;
    const int s = colok ? (int)(col / g.out.P) : 0;
    const int p = colok ? (int)(col - (long)s * g.out.P) : 0;
    const long bicol0 = (long)c0 * g.out.colpad + col;
    // output side: B, P and Q_q per channel
    double Bv[CB], Pv[CB], Q[CB][NM > 0 ? NM : 1];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        Bv[e] = Pv[e] = 0;
#pragma unroll
        for (int q = 0; q < NM; ++q) Q[e][q] = 0;
        if (colok && c0 + e < g.out.C) {
            const long idx_e = ((long)(c0 + e) * S + s) * g.out.P + p;
            const long bo = bicol0 + (long)e * g.out.colpad;
#pragma unroll
            for (int q = 0; q < NM; ++q) {
                const double bq = (double)A.R.slot[q].beta[idx_e];
                Bv[e] += bq;
                if (getbit(A.R.slot[q].zbits, bo)) Pv[e] += bq;
                else Q[e][q] = bq;
            }
        }
    }
    double r1[CB], r0x[CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) r1[e] = r0x[e] = 0;
    const int F = g.fan;
    const int t0 = (int)((long)F * wave / NW), t1 = (int)((long)F * (wave + 1) / NW);
    // one tap: box ends, point-box bit, the masks' x bits (cleared on a point box)
    auto tap = [&](int t, double lo, double hi, unsigned dg, unsigned xb) {
        double xd[NM > 0 ? NM : 1];
#pragma unroll
        for (int q = 0; q < NM; ++q) xd[q] = ((xb >> q) & 1u) ? 1.0 : 0.0;
#pragma unroll
        for (int e = 0; e < CB; ++e) {
            const float wf = c0 + e < g.out.C ? g.W[(long)(c0 + e) * F + t] : 0.f;
            if (wf == 0.f) continue;
            const double w = (double)wf;
            double X = 0;
            if constexpr (NM > 0) {
                X = xd[0] * Q[e][0];
#pragma unroll
                for (int q = 1; q < NM; ++q) X = fma(xd[q], Q[e][q], X);
            }
            if (wf > 0.f) {
                const double PD = Bv[e] - X;
                r1[e] = fma(w * lo, PD, r1[e]);
                r0x[e] = fma(w * hi, Bv[e] - PD, r0x[e]);
            } else {
                const double PD = dg ? Bv[e] : Pv[e] + X;
                r1[e] = fma(w * hi, PD, r1[e]);
                r0x[e] = fma(w * lo, Bv[e] - PD, r0x[e]);
            }
        }
    };
    if (colok) {
        if constexpr (DV) {
            // dense layer: 4 consecutive taps are 4 consecutive records
            for (int t = t0; t < t1; t += 4) {
                const int ci = t / g.in.P, pj = t - ci * g.in.P;
                const long a = ((long)ci * S + s) * g.in.P + pj;
                GwIn<float> v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = rec[a + u];
#pragma unroll
                for (int u = 0; u < 4; ++u) tap(t + u, (double)v[u].l, (double)v[u].u, v[u].bits & 1u, v[u].bits >> 1);
            }
        } else {
            TapWalk tw = tap_walk(g, p, t0);
            for (int t = t0; t < t1; ++t, tap_next(g, tw)) {
                const FwdTap tp = tap_at(g, S, s, tw);
                if (tp.a < 0) continue;
                const GwIn<float> v = rec[tp.a];
                tap(t, (double)v.l, (double)v.u, v.bits & 1u, v.bits >> 1);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        red[((wave * CB + e) * 2 + 0) * kWave + lane] = r1[e] + r0x[e];
        red[((wave * CB + e) * 2 + 1) * kWave + lane] = r1[e];
    }
    __syncthreads();
    const int e = wave;
    if (e >= CB) return;
    const int c = c0 + e;
    if (!colok || c >= g.out.C) return;
    const long idx = ((long)c * S + s) * g.out.P + p;
    double r0 = 0, r1s = 0;
    for (int w = 0; w < NW; ++w) {
        r0 += red[((w * CB + e) * 2 + 0) * kWave + lane];
        r1s += red[((w * CB + e) * 2 + 1) * kWave + lane];
    }
    // own = alpha - beta0 - beta1 - sum beta_I,
    // g = beta0 uhat + beta1 lhat + sum beta_I (LI + UI + b),
    // const = b alpha + beta1 (lhat - b) + sum LI beta_I
    const double bb = (double)g.b[c];
    const double al = A.R.alpha[idx], b0 = A.R.beta0[idx], b1 = A.R.beta1[idx];
    const double lh = A.R.lhat[idx], uh = A.R.uhat[idx];
    double sb = 0;
#pragma unroll
    for (int q = 0; q < NM; ++q) sb += (double)A.R.slot[q].beta[idx];
    A.R.own64[idx] = al - b0 - b1 - sb;
    A.R.g64[idx] = b0 * uh + b1 * lh + r0 + bb * sb;
    A.R.const64[idx] = bb * al + b1 * (lh - bb) + r1s;
}

// FP64 backward pass of the final bound of an FP32 plan (f_k, x*_k, z*_k
// and the objective terms of neuron layer k) in sign classes.  For neuron j
// of layer k and an output o of layer k+1 that reads it with weight w, the
// masked part of f_k[j] is sum_q c_q u_q[o], where u_q = (1 - z_q[o]) b_q and
// c_q is w where mask q contains j (w > 0: x not at the upper end; w < 0: x
// at the upper end; both on a point box).  With U = sum_q u_q and
// Xu = sum_q xbit_q[j] u_q (no point box): w > 0 gives w (U - Xu), w < 0
// gives w (Xu + [point box] U), so a pair costs one FMA per mask plus four,
// written as max(w, 0) (U - Xu) + min(w, 0) (Xu + [point] U).
// Output-side record of one neuron of layer k+1 for the FP64 backward into
// layer k (bf_rec_units 16-byte units): v = -alpha + beta_1 + sum over
// z_q = 1 of b_q and U = sum_q u_q in FP64, then the u_q = (1 - z_q) b_q
// (FP32 values, exact as floats).
template <int NM>
__global__ void __launch_bounds__(256) k_bf_outrec(BwdArgs<float> A, float4* rec) {
    const NeuronLayout& O = A.gn.out;
    const long gid = (long)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (long)O.C * O.cols) return;
    const int co = (int)(gid / O.cols);
    const long bi = (long)co * O.colpad + (gid - (long)co * O.cols);
    double v = -(double)A.Rn.alpha[gid] + (double)A.Rn.beta1[gid], U = 0;
    constexpr int NQ = bf_rec_units(NM) * 4 - 4 > 0 ? bf_rec_units(NM) * 4 - 4 : 1;
    float uq[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) uq[i] = 0.f;
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        const float bq = A.Rn.slot[q].beta[gid];
        if (getbit(A.Rn.slot[q].zbits, bi)) {
            v += (double)bq;
        } else {
            uq[q] = bq;
            U += (double)bq;
        }
    }
    float4* r = rec + gid * bf_rec_units(NM);
    double2 vu;
    vu.x = v;
    vu.y = U;
    *reinterpret_cast<double2*>(r) = vu;
#pragma unroll
    for (int i = 1; i < bf_rec_units(NM); ++i)
        r[i] = make_float4(uq[4 * i - 4], uq[4 * i - 3], uq[4 * i - 2], uq[4 * i - 1]);
}

template <int NM>
__global__ void __launch_bounds__(kWave * KS) k_backward_final_sc(BwdArgs<float> A, const float4* orec) {
    extern __shared__ unsigned char red_raw[];
    double* red = reinterpret_cast<double*>(red_raw);  // [KS][CB][64]
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;   // layer k
    const NeuronLayout& O = g.out;  // layer k+1
    const int lane = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S;
    const bool colok = col < L.cols;
    const int s = colok ? (int)(col / L.P) : 0;
    const int p = colok ? (int)(col - (long)s * L.P) : 0;
    // per channel: point-box bit, the masks' x bits as 0/1 (none on a point box)
    unsigned dg4 = 0;
    double xd[CB][NM > 0 ? NM : 1], dgd[CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        dgd[e] = 0;
#pragma unroll
        for (int q = 0; q < NM; ++q) xd[e][q] = 0;
        if (colok && c0 + e < L.C) {
            const long bie = (long)(c0 + e) * L.colpad + col;
            const unsigned dg = getbit(A.nk.deg, bie);
            dg4 |= dg << e;
            dgd[e] = dg ? 1.0 : 0.0;
            if (!dg)
#pragma unroll
                for (int q = 0; q < NM; ++q) xd[e][q] = getbit(A.Rn.slot[q].xbits, bie) ? 1.0 : 0.0;
        }
    }
    double acc[CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) acc[e] = 0;
    // output o at neuron address a (bit index bi) with the weights w[e] to
    // this lane's channels
    auto add_output = [&](long a, long bi, const double* w) {
        double v, uq[NM > 0 ? NM : 1], U = 0;
        if (A.last) {
            v = -(double)A.cvec[a];
#pragma unroll
            for (int q = 0; q < NM; ++q) uq[q] = 0;
        } else {
            // the output's record (k_bf_outrec)
            const float4* r = orec + a * bf_rec_units(NM);
            const double2 vu = *reinterpret_cast<const double2*>(r);
            v = vu.x;
            U = vu.y;
#pragma unroll
            for (int i = 1; i < bf_rec_units(NM); ++i) {
                const float4 f = r[i];
                const float fq[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (4 * i - 4 + j < NM) uq[4 * i - 4 + j] = (double)fq[j];
            }
        }
        (void)bi;
#pragma unroll
        for (int e = 0; e < CB; ++e) {
            double Xu = 0;
            if constexpr (NM > 0) {
                Xu = xd[e][0] * uq[0];
#pragma unroll
                for (int q = 1; q < NM; ++q) Xu = fma(xd[e][q], uq[q], Xu);
            }
            acc[e] = fma(w[e], v, acc[e]);
            acc[e] = fma(fmax(w[e], 0.0), U - Xu, acc[e]);
            acc[e] = fma(fmin(w[e], 0.0), fma(dgd[e], U, Xu), acc[e]);
        }
    };
    if (colok) {
        if (g.kind == ASD_LAYER_DENSE) {
            const int n1 = O.C;
            const int i0 = (int)((long)n1 * wave / KS), i1 = (int)((long)n1 * (wave + 1) / KS);
            for (int i = i0; i < i1; ++i) {
                double w[CB];
#pragma unroll
                for (int e = 0; e < CB; ++e)
                    w[e] = c0 + e < L.C ? (double)g.W[(long)i * g.fan + (long)(c0 + e) * L.P + p] : 0.0;
                add_output((long)i * S + s, (long)i * O.colpad + s, w);
            }
        } else {
            const int y = p / L.W, x = p - (p / L.W) * L.W;
            const int co0 = (int)((long)O.C * wave / KS), co1 = (int)((long)O.C * (wave + 1) / KS);
            const int ks = g.ksz, str = g.stride;
            const int ky0 = (y + g.pad) % str, kx0 = (x + g.pad) % str;
            const int oyf = (y + g.pad - ky0) / str, oxf = (x + g.pad - kx0) / str;
            for (int co = co0; co < co1; ++co) {
                int oy = oyf;
                for (int ky = ky0; ky < ks; ky += str, --oy) {
                    if (oy < 0 || oy >= O.H) continue;
                    int ox = oxf;
                    for (int kx = kx0; kx < ks; kx += str, --ox) {
                        if (ox < 0 || ox >= O.W) continue;
                        const int op = oy * O.W + ox;
                        double w[CB];
#pragma unroll
                        for (int e = 0; e < CB; ++e)
                            w[e] = c0 + e < L.C ? (double)g.W[(((long)co * L.C + c0 + e) * ks + ky) * ks + kx] : 0.0;
                        add_output(((long)co * S + s) * O.P + op, (long)co * O.colpad + (long)s * O.P + op, w);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < CB; ++e) red[(wave * CB + e) * kWave + lane] = acc[e];
    __syncthreads();
    const int e = wave;
    const int c = c0 + e;
    if (c >= L.C) return;  // whole wave leaves together
    const long idx = ((long)c * S + s) * L.P + p;
    bool xb = false, zb = false;
    if (colok) {
        double f = 0;
        for (int w = 0; w < KS; ++w) f += red[(w * CB + e) * kWave + lane];
        if (A.k >= 1) f += A.Rk.own64[idx];
        if (A.fout) A.fout[idx] = f;
        if (A.fext) A.fext[(long)s * L.N + (long)c * L.P + p] = (float)f;
        // x-bit "x* = upper end"; a point box counts as both ends and keeps the bit set
        xb = f >= 0 || ((dg4 >> e) & 1u);
        const double xv = xb ? (double)A.nk.hi[idx] : (double)A.nk.lo[idx];
        A.nk.xstar[idx] = (float)xv;
        double term = -f * xv;
        if (A.k >= 1) {
            const double gk = A.Rk.g64[idx];
            zb = gk >= 0;
            term -= zb ? gk : 0.0;
            if (A.want_obj) term += A.Rk.const64[idx];
        }
        if (A.want_obj) A.nk.term[idx] = term;
    }
    const long base = (long)c * L.colpad + (long)blockIdx.x * kWave;
    put_wave_bits(A.nk.xbits, base, colok && xb, lane);
    if (A.k >= 1) put_wave_bits(A.Rk.zbits, base, colok && zb, lane);
}

}  // namespace

template <int NM>
asd_status final_sums_nm(asd_plan* P, int k, void* inrec, hipStream_t st) {
    const LayerGeo& g = P->geo[k];
    // input records of layer k-1 (box ends, point-box and x bits)
    GradArgs<float> ga;
    memset(&ga, 0, sizeof(ga));
    ga.g = g;
    ga.S = P->S;
    ga.nm = NM;
    ga.xin = P->naf[k - 1].xstar;
    ga.lo_in = P->naf[k - 1].lo;
    ga.hi_in = P->naf[k - 1].hi;
    ga.deg_in = P->naf[k - 1].deg;
    ga.R = RdevT<float>(P) + k;
    GwIn<float>* rec = static_cast<GwIn<float>*>(inrec);
    const long nin = (long)g.in.C * g.in.cols;
    hipLaunchKernelGGL(k_gw_in<float>, dim3((unsigned)((nin + kGradThreads - 1) / kGradThreads)), dim3(kGradThreads),
                       0, st, ga, rec);
    LAUNCH_CHECK();
    MaskArgs<float> a;
    memset(&a, 0, sizeof(a));
    a.g = g;
    a.S = P->S;
    a.nm = NM;
    a.R = P->Rf[k];
    const dim3 grid = grid_cols(P->nl[k], CB);
    const bool dv16 = g.kind == ASD_LAYER_DENSE && g.in.P % 4 == 0 && g.fan % (4 * 16) == 0;
    const bool dv4 = g.kind == ASD_LAYER_DENSE && g.in.P % 4 == 0 && g.fan % (4 * KS) == 0;
    if (g.fan >= 1024) {
        const size_t lds = (size_t)16 * CB * 2 * kWave * sizeof(double);
        if (dv16) hipLaunchKernelGGL((k_final_sums_sc<NM, 16, true>), grid, dim3(kWave, 16), lds, st, a, rec);
        else hipLaunchKernelGGL((k_final_sums_sc<NM, 16, false>), grid, dim3(kWave, 16), lds, st, a, rec);
    } else {
        const size_t lds = (size_t)KS * CB * 2 * kWave * sizeof(double);
        if (dv4) hipLaunchKernelGGL((k_final_sums_sc<NM, KS, true>), grid, dim3(kWave, KS), lds, st, a, rec);
        else hipLaunchKernelGGL((k_final_sums_sc<NM, KS, false>), grid, dim3(kWave, KS), lds, st, a, rec);
    }
    LAUNCH_CHECK();
    return ASD_OK;
}

template <int NM>
asd_status backward_final_nm(const BwdArgs<float>& a, void* orec, hipStream_t st) {
    float4* rec = static_cast<float4*>(orec);
    if (!a.last) {
        const long nout = (long)a.gn.out.C * a.gn.out.cols;
        hipLaunchKernelGGL((k_bf_outrec<NM>), dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, st, a, rec);
        LAUNCH_CHECK();
    }
    const size_t lds = (size_t)KS * CB * kWave * sizeof(double);
    hipLaunchKernelGGL((k_backward_final_sc<NM>), grid_cols(a.gn.in, CB), dim3(kWave, KS), lds, st, a,
                       (const float4*)rec);
    LAUNCH_CHECK();
    return ASD_OK;
}

template asd_status final_sums_nm<ASD_NM>(asd_plan*, int, void*, hipStream_t);
template asd_status backward_final_nm<ASD_NM>(const BwdArgs<float>&, void*, hipStream_t);

}  // namespace asd
