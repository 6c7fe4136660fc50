// Launches of the ReLU-layer weight-gradient and box-gradient kernels
// (asd_adjoint.h) for one count of active masks: this file is compiled once per count with
// -DASD_NM=<count>, so the kernels of the different counts build in parallel.
#include "asd_adjoint.h"
#include "asd_plan.h"

#ifndef ASD_NM
#error "compile with -DASD_NM=<active mask count>"
#endif

namespace asd {

template <typename Ts, int NM>
asd_status gw_relu_t(asd_plan* P, int k, const double* gs, const void* inrec, hipStream_t st) {
    const LayerGeo& g = P->geo[k];
    GwArgs<Ts> a;
    memset(&a, 0, sizeof(a));
    a.S = P->S;
    a.fan = g.fan;
    if (g.kind == ASD_LAYER_DENSE) {
        // a dense layer is a convolution whose kernel covers the whole input
        a.kh = g.in.H;
        a.kw = g.in.W;
        a.stride = 1;
        a.pad = 0;
    } else {
        a.kh = a.kw = g.ksz;
        a.stride = g.stride;
        a.pad = g.pad;
    }
    a.inH = g.in.H;
    a.inW = g.in.W;
    a.inP = g.in.P;
    a.outC = g.out.C;
    a.outH = g.out.H;
    a.outW = g.out.W;
    a.outP = g.out.P;
    a.outcols = g.out.cols;
    a.outcolpad = g.out.colpad;
    a.W = g.W;
    a.gs = gs;
    a.in = static_cast<const GwIn<Ts>*>(inrec);
    a.R = RdevT<Ts>(P) + k;
    a.r_chunk = P->gw_rchunk[k];
    a.entries = (long)g.out.C * g.fan;
    a.part = P->gpart;
    int TT, TO;
    gw_config(g.fan, &TT, &TO);
    const dim3 grid((unsigned)P->gw_chunks[k], (unsigned)((g.fan + 64 * TT - 1) / (64 * TT)),
                    (unsigned)((g.out.C + TO - 1) / TO));
    if (TT == 1) hipLaunchKernelGGL((k_gw_relu<Ts, NM, 8, 1>), grid, dim3(kGradThreads), 0, st, a);
    else if (TT == 2) hipLaunchKernelGGL((k_gw_relu<Ts, NM, 4, 2>), grid, dim3(kGradThreads), 0, st, a);
    else hipLaunchKernelGGL((k_gw_relu<Ts, NM, 4, 4>), grid, dim3(kGradThreads), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

// Box gradient through layer 1 with the sign-class kernel; *done stays false
// where it does not apply (no active mask, or LDS too small for its records).
template <typename Ts, int NM>
asd_status grad_box_t(asd_plan* P, const double* gs, double* dl0, double* du0, bool* done, hipStream_t st) {
    const LayerGeo& g = P->geo[1];
    if (NM == 0 || P->n < 2) return ASD_OK;
    const int NC = std::max(1, std::min(g.out.C, 256 / g.out.P));
    const size_t lds = grad_box_lds(g, NM, NC);
    if (lds > 65536) return ASD_OK;
    GradArgs<Ts> a;
    memset(&a, 0, sizeof(a));
    a.g = g;
    a.S = P->S;
    a.nm = NM;
    a.gs = gs;
    a.deg_in = NA<Ts>(P)[0].deg;
    a.R = RdevT<Ts>(P) + 1;
    a.f0 = P->f0;
    a.dl0 = dl0;
    a.du0 = du0;
    const dim3 grid((unsigned)((g.in.N + kGradThreads * kGbNI - 1) / (kGradThreads * kGbNI)), (unsigned)P->S);
    if (g.kind == ASD_LAYER_DENSE)
        hipLaunchKernelGGL((k_grad_box_sc<Ts, NM, true>), grid, dim3(kGradThreads), lds, st, a, NC);
    else
        hipLaunchKernelGGL((k_grad_box_sc<Ts, NM, false>), grid, dim3(kGradThreads), lds, st, a, NC);
    LAUNCH_CHECK();
    *done = true;
    return ASD_OK;
}

template <int NM>
asd_status grad_box_nm(asd_plan* P, const double* gs, double* dl0, double* du0, bool* done, hipStream_t st) {
    return is64(P) ? grad_box_t<double, NM>(P, gs, dl0, du0, done, st)
                   : grad_box_t<float, NM>(P, gs, dl0, du0, done, st);
}

template <int NM>
asd_status grad_weight_nm(asd_plan* P, int k, const double* gs, const void* inrec, hipStream_t st) {
    return is64(P) ? gw_relu_t<double, NM>(P, k, gs, inrec, st) : gw_relu_t<float, NM>(P, k, gs, inrec, st);
}

template asd_status grad_weight_nm<ASD_NM>(asd_plan*, int, const double*, const void*, hipStream_t);
template asd_status grad_box_nm<ASD_NM>(asd_plan*, const double*, double*, double*, bool*, hipStream_t);

}  // namespace asd
