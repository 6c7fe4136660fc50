// Launches of the iteration kernels (asd_fast.h) for one count of active
// masks: this file is compiled once per count with -DASD_NM=<count>, so the
// kernels of the different counts build in parallel.
#include "asd_plan.h"

#ifndef ASD_NM
#error "compile with -DASD_NM=<active mask count>"
#endif

namespace asd {

// Iteration forward pass of ReLU layer k with NM active masks.
template <typename T, int NM, bool MB, bool BF>
asd_status fwd_fast_impl(asd_plan* P, int k, const StepArgsT<T>& sa, hipStream_t st) {
    FastFwdArgs<T> a = fwd_args<T>(P, k, NM, sa);
    const LayerGeo& g = a.g;
    constexpr int CB = sizeof(T) == 4 ? 8 : 4;
    ProfScope ps(P, st, ASD_K_FORWARD, k);
    if (g.kind == ASD_LAYER_CONV2D && !P->fwd_mfma[k]) {
        // narrow layer: a 32-row matrix tile would be half empty, and the
        // update's memory traffic bounds it anyway
        dim3 grid((unsigned)((g.out.cols + kWave - 1) / kWave), (unsigned)((g.out.C + CB - 1) / CB));
        if (g.ksz == 4)
            hipLaunchKernelGGL((k_fwd_conv<T, NM, CB, 4, MB>), grid, dim3(kWave, KS), 0, st, a);
        else
            hipLaunchKernelGGL((k_fwd_conv<T, NM, CB, 0, MB>), grid, dim3(kWave, KS), 0, st, a);
        LAUNCH_CHECK();
        return ASD_OK;
    }
    if (g.kind == ASD_LAYER_CONV2D) {
        // one 32-column tile per block, its waves splitting the taps
        const long ntiles = (g.out.cols + 31) / 32;
        dim3 grid((unsigned)ntiles, (unsigned)(a.Cpad / 32));
        if (P->fwd_kw[k] == 8) {
            if (g.ksz == 4) hipLaunchKernelGGL((k_fwd_conv_mfma<NM, true, 4, MB, 8, BF>), grid, dim3(kWave, 8), 0, st, a);
            else hipLaunchKernelGGL((k_fwd_conv_mfma<NM, true, 0, MB, 8, BF>), grid, dim3(kWave, 8), 0, st, a);
        } else {
            if (g.ksz == 4) hipLaunchKernelGGL((k_fwd_conv_mfma<NM, true, 4, MB, 4, BF>), grid, dim3(kWave, 4), 0, st, a);
            else hipLaunchKernelGGL((k_fwd_conv_mfma<NM, true, 0, MB, 4, BF>), grid, dim3(kWave, 4), 0, st, a);
        }
        (void)CB;
        LAUNCH_CHECK();
        return ASD_OK;
    }
    dim3 grid((unsigned)((P->Sa + 31) / 32), (unsigned)(a.Cpad / 32), (unsigned)a.ksplit);
    if (a.ksplit == 1) {
        // one split: the product blocks update their neurons themselves
        if (P->fwd_kw[k] == 8) hipLaunchKernelGGL((k_fwd_dense_mfma<NM, 8, true, MB, BF>), grid, dim3(kWave, 8), 0, st, a);
        else hipLaunchKernelGGL((k_fwd_dense_mfma<NM, 4, true, MB, BF>), grid, dim3(kWave, 4), 0, st, a);
        LAUNCH_CHECK();
        return ASD_OK;
    }
    if (P->fwd_kw[k] == 8) hipLaunchKernelGGL((k_fwd_dense_mfma<NM, 8, false, MB, BF>), grid, dim3(kWave, 8), 0, st, a);
    else hipLaunchKernelGGL((k_fwd_dense_mfma<NM, 4, false, MB, BF>), grid, dim3(kWave, 4), 0, st, a);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_fwd_dense_epi<T, NM, MB>), dim3((unsigned)((P->Sa + 255) / 256), (unsigned)g.out.C), dim3(256),
                       0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <int NM>
asd_status fwd_fast_nm(asd_plan* P, int k, const StepArgsT<float>& sa, bool mb, hipStream_t st) {
    if (bf16_forward(P)) return fwd_fast_impl<float, NM, true, true>(P, k, sa, st);
    return mb ? fwd_fast_impl<float, NM, true, false>(P, k, sa, st) : fwd_fast_impl<float, NM, false, false>(P, k, sa, st);
}

// The forward pass of convolutional layer kc on the matrix cores (8 waves
// per tile) and the products of dense layer kd (8 waves per split) in one
// launch (k_fwd_conv_dense), then the dense layer's epilogue.
template <int NM, bool MB, bool BF>
asd_status fwd_fused_impl(asd_plan* P, int kc, int kd, const StepArgsT<float>& sa, hipStream_t st) {
    const FastFwdArgs<float> ac = fwd_args<float>(P, kc, NM, sa);
    const FastFwdArgs<float> ad = fwd_args<float>(P, kd, NM, sa);
    const int dgx = (P->Sa + 31) / 32, dgy = ad.Cpad / 32, nd = dgx * dgy * ad.ksplit;
    const int cgx = (int)((ac.g.out.cols + 31) / 32), cgy = ac.Cpad / 32;
    const dim3 grid((unsigned)(nd + cgx * cgy));
    const bool du = ad.ksplit == 1;  // one split: the dense blocks update, no epilogue
    ProfScope ps(P, st, ASD_K_FORWARD_PASS, std::min(kc, kd));
    if (ac.g.ksz == 4) {
        if (du) hipLaunchKernelGGL((k_fwd_conv_dense<NM, 4, MB, true, BF>), grid, dim3(kWave, 8), 0, st, ac, ad, nd, dgx, dgy, cgx, cgy);
        else hipLaunchKernelGGL((k_fwd_conv_dense<NM, 4, MB, false, BF>), grid, dim3(kWave, 8), 0, st, ac, ad, nd, dgx, dgy, cgx, cgy);
    } else {
        if (du) hipLaunchKernelGGL((k_fwd_conv_dense<NM, 0, MB, true, BF>), grid, dim3(kWave, 8), 0, st, ac, ad, nd, dgx, dgy, cgx, cgy);
        else hipLaunchKernelGGL((k_fwd_conv_dense<NM, 0, MB, false, BF>), grid, dim3(kWave, 8), 0, st, ac, ad, nd, dgx, dgy, cgx, cgy);
    }
    LAUNCH_CHECK();
    if (du) return ASD_OK;
    hipLaunchKernelGGL((k_fwd_dense_epi<float, NM, MB>), dim3((unsigned)((P->Sa + 255) / 256), (unsigned)ad.g.out.C),
                       dim3(256), 0, st, ad);
    LAUNCH_CHECK();
    return ASD_OK;
}

// The forward pass of VALU-mapped convolutional layer kv, matrix-core
// convolutional layer kc and dense layer kd in one launch (k_fwd_trio), then
// the dense layer's epilogue.
template <int NM, bool MB, bool BF>
asd_status fwd_trio_impl(asd_plan* P, int kv, int kc, int kd, const StepArgsT<float>& sa, hipStream_t st) {
    const FastFwdArgs<float> av = fwd_args<float>(P, kv, NM, sa);
    const FastFwdArgs<float> ac = fwd_args<float>(P, kc, NM, sa);
    const FastFwdArgs<float> ad = fwd_args<float>(P, kd, NM, sa);
    const int dgx = (P->Sa + 31) / 32, dgy = ad.Cpad / 32, nd = dgx * dgy * ad.ksplit;
    const int cgx = (int)((ac.g.out.cols + 31) / 32), cgy = ac.Cpad / 32, nc = cgx * cgy;
    const int vgx = (int)((av.g.out.cols + kWave - 1) / kWave), vgy = (av.g.out.C + 7) / 8;
    const int nv = (vgx * vgy + 1) / 2;  // two column-kernel blocks per launched block
    // the convolutions' blocks in order (matrix-core ones first): measured
    // faster than interleaving them
    const int ip = 1;
    const dim3 grid((unsigned)(nd + nc + nv));
    const bool c4 = ac.g.ksz == 4, v4 = av.g.ksz == 4;
    const bool du = ad.ksplit == 1;  // one split: the dense blocks update, no epilogue
    ProfScope ps(P, st, ASD_K_FORWARD_PASS, std::min(kv, std::min(kc, kd)));
#define ASD_TRIO_LAUNCH(KC, KV)                                                                                       \
    do {                                                                                                              \
        if (du)                                                                                                       \
            hipLaunchKernelGGL((k_fwd_trio<NM, KC, KV, MB, true, BF>), grid, dim3(kWave, 8), 0, st, av, ac, ad, nd, dgx, \
                               dgy, nc, cgx, cgy, vgx, vgy, ip);                                                      \
        else                                                                                                          \
            hipLaunchKernelGGL((k_fwd_trio<NM, KC, KV, MB, false, BF>), grid, dim3(kWave, 8), 0, st, av, ac, ad, nd, dgx, \
                               dgy, nc, cgx, cgy, vgx, vgy, ip);                                                      \
    } while (0)
    if (c4 && v4) ASD_TRIO_LAUNCH(4, 4);
    else if (c4) ASD_TRIO_LAUNCH(4, 0);
    else if (v4) ASD_TRIO_LAUNCH(0, 4);
    else ASD_TRIO_LAUNCH(0, 0);
#undef ASD_TRIO_LAUNCH
    LAUNCH_CHECK();
    if (du) return ASD_OK;
    hipLaunchKernelGGL((k_fwd_dense_epi<float, NM, MB>), dim3((unsigned)((P->Sa + 255) / 256), (unsigned)ad.g.out.C),
                       dim3(256), 0, st, ad);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <int NM>
asd_status fwd_fused_nm(asd_plan* P, int kc, int kd, const StepArgsT<float>& sa, bool mb, hipStream_t st) {
    if (bf16_forward(P)) return fwd_fused_impl<NM, true, true>(P, kc, kd, sa, st);
    return mb ? fwd_fused_impl<NM, true, false>(P, kc, kd, sa, st) : fwd_fused_impl<NM, false, false>(P, kc, kd, sa, st);
}

template <int NM>
asd_status fwd_trio_nm(asd_plan* P, int kv, int kc, int kd, const StepArgsT<float>& sa, bool mb, hipStream_t st) {
    if (bf16_forward(P)) return fwd_trio_impl<NM, true, true>(P, kv, kc, kd, sa, st);
    return mb ? fwd_trio_impl<NM, true, false>(P, kv, kc, kd, sa, st)
              : fwd_trio_impl<NM, false, false>(P, kv, kc, kd, sa, st);
}

template <int NM, bool BF>
asd_status bwd_pair_impl(asd_plan* P, hipStream_t st) {
    const int ka = P->n - 1, kb = P->n - 2;
    const FastBwdArgs<float> aa = bwd_args<float>(P, ka, 0);
    const FastBwdArgs<float> ab = bwd_args<float>(P, kb, NM);
    const NeuronLayout& La = aa.gn.in;
    const NeuronLayout& Lb = ab.gn.in;
    const int agx = (int)((La.cols + kWave - 1) / kWave), agy = (La.C + 7) / 8, na = agx * agy;
    const int mgx = (P->Sa + 15) / 16, mgy = Lb.C * (Lb.P / kWave);
    ProfScope ps(P, st, ASD_K_BACKWARD_PAIR, kb);
    hipLaunchKernelGGL((k_bwd_dense_pair<NM, BF>), dim3((unsigned)(na + mgx * mgy)), dim3(kWave, 4), 0, st, aa, ab, na, agx,
                       agy, mgx);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <int NM>
asd_status bwd_pair_nm(asd_plan* P, hipStream_t st) {
    return bf16_backward(P) ? bwd_pair_impl<NM, true>(P, st) : bwd_pair_impl<NM, false>(P, st);
}

// Iteration backward pass into neuron layer k; NM = masks of layer k+1.
template <int NM, bool BF>
asd_status bwd_fast_impl(asd_plan* P, int k, hipStream_t st) {
    using T = float;
    FastBwdArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.gn = gview(P, k + 1);
    a.S = P->S;
    a.k = k;
    a.last = (k + 1 == P->n);
    a.nm = NM;
    a.Wr = P->Wr[k + 1];
    a.fanpad = P->fanpad[k + 1];
    a.cvec = CV<T>(P);
    if (!a.last) {
        const ReluLayerT<T>& rn = RL<T>(P)[k + 1];
        a.vs = rn.vs;
        for (int q = 0; q < NM; ++q) a.u[q] = rn.slot[q].u;
    } else {
        a.vs = P->negc;  // a convolutional output layer's operand (dense ones read cvec)
    }
    a.xpk = NA<T>(P)[k].xpk;
    a.nk = NA<T>(P)[k];
    if (k >= 1) {
        const ReluLayerT<T>& r = RL<T>(P)[k];
        a.own = r.own;
        a.gk = r.g;
        a.zbits = r.zbits;
    }
    const LayerGeo& g = a.gn;
    const NeuronLayout& L = g.in;
    a.Wb = P->Wb[k + 1];
    a.Wl4 = P->Wl4[k + 1];
    a.Wl8 = P->Wl8[k + 1];
    a.nkp = P->nkp[k + 1];
    a.fout = reinterpret_cast<T*>(P->ev_f[k]);
    if (k == 0 && P->domain == ASD_DOMAIN_L2 && !a.fout) a.fout = P->f0f;  // f_0 for the ball's x*_0
    if (g.kind == ASD_LAYER_CONV2D && L.P % kWave == 0 && L.C >= 16) {
        // matrix-core transposed convolution over parity classes, operands
        // staged in LDS (see k_bwd_conv_mfma); shapes it cannot hold fall
        // through to the column kernel
        BwdConvShape sh = conv_shape(g);
        const int st_ = g.stride, pd = g.pad;
        // items of NT column tiles of 16 positions of one parity class; one
        // wave per item, at most 8: two tiles per item where that fits
        auto count_items = [&](int nt) {
            int items = 0;
            for (int c = 0; c < st_ * st_; ++c) {
                const int ry = c / st_, rx = c % st_;
                const int yf = ((ry - pd) % st_ + st_) % st_, xf = ((rx - pd) % st_ + st_) % st_;
                const int ny = yf < L.H ? (L.H - 1 - yf) / st_ + 1 : 0;
                const int nx = xf < L.W ? (L.W - 1 - xf) / st_ + 1 : 0;
                items += (ny * nx + 16 * nt - 1) / (16 * nt);
            }
            return items;
        };
        const int NT = (count_items(2) <= 8 && P->bwd_nt[k] != 4) ? 2 : 4;
        sh.items = count_items(NT);
        sh.NW = std::min(sh.items, 8);
        const size_t fbytes = (size_t)std::min(16, L.C) * L.P * sizeof(float);
        constexpr int RS = bwd_mfma_rs<NM>();
        const int img = sh.Hp * sh.Wp;
        if (sh.items <= sh.NW && fbytes <= 32 * 1024 && img <= RS) {
            sh.CC = std::min(g.out.C, RS / img);
            // product r's images at float r RS, the parked f after the last;
            // or (wl) the class weights after the last image and f parked
            // over the images, where two blocks per CU still fit
            const int fbo4 = (NM * RS + sh.CC * img + 3) / 4 * 4;
            const size_t wfl = (size_t)st_ * st_ * a.nkp * 16;
            const bool wl = g.ksz == 4 && g.stride == 2 && NT == 2 && sh.CC == g.out.C &&
                            fbytes <= (size_t)(NM * RS + sh.CC * img) * sizeof(float) &&
                            ((size_t)fbo4 + wfl) * sizeof(float) <= std::min<size_t>((size_t)P->lds_max, 80 * 1024);
            sh.fboff = wl ? fbo4 : NM * RS + sh.CC * img;
            const size_t dyn = wl ? ((size_t)fbo4 + wfl) * sizeof(float) : (size_t)sh.fboff * sizeof(float) + fbytes;
            ProfScope ps(P, st, ASD_K_BACKWARD, k);
            dim3 grid((unsigned)P->Sa, (unsigned)((L.C + 15) / 16));
            if (g.ksz == 4 && g.stride == 2) {
                if (wl) hipLaunchKernelGGL((k_bwd_conv_mfma<NM, 4, 2, 2, BF, true>), grid, dim3(kWave, sh.NW), dyn, st, a, sh);
                else if (NT == 2) hipLaunchKernelGGL((k_bwd_conv_mfma<NM, 4, 2, 2, BF>), grid, dim3(kWave, sh.NW), dyn, st, a, sh);
                else hipLaunchKernelGGL((k_bwd_conv_mfma<NM, 4, 2, 4, BF>), grid, dim3(kWave, sh.NW), dyn, st, a, sh);
            } else {
                if (NT == 2) hipLaunchKernelGGL((k_bwd_conv_mfma<NM, 0, 0, 2>), grid, dim3(kWave, sh.NW), dyn, st, a, sh);
                else hipLaunchKernelGGL((k_bwd_conv_mfma<NM, 0, 0, 4>), grid, dim3(kWave, sh.NW), dyn, st, a, sh);
            }
            LAUNCH_CHECK();
            return ASD_OK;
        }
    }
    if (g.kind == ASD_LAYER_CONV2D) {
        // column kernel, the taps split over KS waves
        const int CB = (sizeof(T) == 4 && L.C > 4 && P->bwd_cb[k] != 4) ? 8 : 4;
        const int ksp = KS;
        const size_t dyn = ((size_t)g.out.C * g.ksz * g.ksz + 1) * CB * sizeof(float);  // + a zero row
        const size_t stat = (size_t)ksp * CB * kWave * sizeof(T);
        if (dyn + stat > 64 * 1024) return launch_backward_iter(P, k, st);
        ProfScope ps(P, st, ASD_K_BACKWARD, k);
        dim3 grid((unsigned)((L.cols + kWave - 1) / kWave), (unsigned)((L.C + CB - 1) / CB));
        const bool k4s2 = g.ksz == 4 && g.stride == 2;
        if constexpr (sizeof(T) == 4) {
            if (bwd_m4_fits(P, k) && P->bwd_cb[k] != 4) {
                // at most 4 channels, stride 2: the matrix-core variant, a
                // block per subproblem
                BwdConvShape sh = conv_shape(g);
                const int img = sh.Hp * sh.Wp;
                const int wfl = (g.out.C * g.ksz * g.ksz + 1) * 4;  // weights and the zero row
                // staged images: the LDS share of two blocks per CU where the
                // device and the weights allow, else the 48 KB split
                const bool big = P->lds_max >= 78 * 1024 && wfl <= kM4BigWeightFloats;
                const int RS = big ? bwd_m4_rs_big<NM>() : bwd_mfma_rs<NM>();
                sh.CC = std::min(g.out.C, RS / img);
                sh.fboff = (NM * RS + sh.CC * img + 3) / 4 * 4;
                const size_t dm4 = ((size_t)sh.fboff + (size_t)wfl) * sizeof(float);
                if (dm4 <= (size_t)P->lds_max) {
                    const dim3 bm4(kWave, L.P / kWave);
                    const dim3 gm4((unsigned)P->Sa);
                    if (g.ksz == 4) {
                        if (big) hipLaunchKernelGGL((k_bwd_conv_m4<NM, 4, BF, true>), gm4, bm4, dm4, st, a, sh);
                        else hipLaunchKernelGGL((k_bwd_conv_m4<NM, 4, BF, false>), gm4, bm4, dm4, st, a, sh);
                    } else {
                        if (big) hipLaunchKernelGGL((k_bwd_conv_m4<NM, 0, false, true>), gm4, bm4, dm4, st, a, sh);
                        else hipLaunchKernelGGL((k_bwd_conv_m4<NM, 0, false, false>), gm4, bm4, dm4, st, a, sh);
                    }
                    LAUNCH_CHECK();
                    return ASD_OK;
                }
            }
            if (CB == 8) {
                if (k4s2)
                    hipLaunchKernelGGL((k_bwd_conv<T, NM, 8, 4, 2, KS>), grid, dim3(kWave, KS), dyn, st, a);
                else
                    hipLaunchKernelGGL((k_bwd_conv<T, NM, 8, 0, 0, KS>), grid, dim3(kWave, KS), dyn, st, a);
                LAUNCH_CHECK();
                return ASD_OK;
            }
        }
        if (k4s2)
            hipLaunchKernelGGL((k_bwd_conv<T, NM, 4, 4, 2, KS>), grid, dim3(kWave, KS), dyn, st, a);
        else
            hipLaunchKernelGGL((k_bwd_conv<T, NM, 4, 0, 0, KS>), grid, dim3(kWave, KS), dyn, st, a);
        LAUNCH_CHECK();
        return ASD_OK;
    }
    ProfScope ps(P, st, ASD_K_BACKWARD, k);
    constexpr int SB = sizeof(T) == 4 ? 8 : 4;
    if constexpr (sizeof(T) == 4) {
        if (L.P % kWave == 0 && P->bwd_pos[k] == 2) {
            // matrix cores: 16 subproblems x 64 positions per block
            dim3 grid((unsigned)((P->Sa + 15) / 16), (unsigned)(L.C * (L.P / kWave)));
            hipLaunchKernelGGL((k_bwd_dense_mfma<NM, BF>), grid, dim3(kWave, 4), 0, st, a);
            LAUNCH_CHECK();
            return ASD_OK;
        }
    }
    if (L.P % kWave == 0 && P->S >= SB && P->bwd_pos[k]) {
        dim3 grid((unsigned)(L.C * (L.P / kWave)), (unsigned)((P->Sa + SB - 1) / SB));
        bool done = false;
        if constexpr (SB % 8 == 0) {
            if (P->bwd_kw[k] == 8) {
                hipLaunchKernelGGL((k_bwd_dense_pos<T, NM, SB, 8>), grid, dim3(kWave, 8), 0, st, a);
                done = true;
            }
        }
        if (!done) hipLaunchKernelGGL((k_bwd_dense_pos<T, NM, SB, 4>), grid, dim3(kWave, 4), 0, st, a);
    } else {
        constexpr int CB = sizeof(T) == 4 ? 8 : 4;
        dim3 grid((unsigned)((L.cols + kWave - 1) / kWave), (unsigned)((L.C + CB - 1) / CB));
        if (L.P == 1)
            hipLaunchKernelGGL((k_bwd_dense<T, NM, CB, true>), grid, dim3(kWave, KS), 0, st, a);
        else
            hipLaunchKernelGGL((k_bwd_dense<T, NM, CB, false>), grid, dim3(kWave, KS), 0, st, a);
    }
    LAUNCH_CHECK();
    return ASD_OK;
}

template <int NM>
asd_status bwd_fast_nm(asd_plan* P, int k, hipStream_t st) {
    return bf16_backward(P) ? bwd_fast_impl<NM, true>(P, k, st) : bwd_fast_impl<NM, false>(P, k, st);
}

template asd_status fwd_fast_nm<ASD_NM>(asd_plan*, int, const StepArgsT<float>&, bool, hipStream_t);
template asd_status fwd_fused_nm<ASD_NM>(asd_plan*, int, int, const StepArgsT<float>&, bool, hipStream_t);
template asd_status fwd_trio_nm<ASD_NM>(asd_plan*, int, int, int, const StepArgsT<float>&, bool, hipStream_t);
template asd_status bwd_pair_nm<ASD_NM>(asd_plan*, hipStream_t);
template asd_status bwd_fast_nm<ASD_NM>(asd_plan*, int, hipStream_t);

}  // namespace asd
