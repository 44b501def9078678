// Host implementation of the learned-bracket network entry points of the C
// ABI: creation, forward / gradient / Adam, training loop and prediction.
// The arithmetic runs in the kernels of mlp.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mlp_net.h"
#include "spec.h"
#include "spec_diag.h"

using namespace spec;

void spec_mlp_s::free_work() {
    dfree(dX);
    for (int l = 0; l < MLP_MAX_LAYERS; ++l) {
        dfree(dH[l]);
        dfree(dZ[l]);
    }
    dfree(dY); dfree(dDY); dfree(dD0); dfree(dD1); dfree(dT); dfree(dIdx); dfree(dLoss);
    cap = 0;
}

spec_status spec_mlp_s::ensure(int rows, hipStream_t s) {
    if (rows <= cap) return SPEC_OK;
    free_work();
    const int c = round_up(std::max(rows, 64), 64);
    HIPCHK(dalloc(&dX, (size_t)c * ld_in()));
    for (int l = 0; l < hidden; ++l) {
        HIPCHK(dalloc(&dH[l], (size_t)c * ld_h()));
        HIPCHK(dalloc(&dZ[l], (size_t)c * width, false));
        HIPCHK(mlp_fill_col(c, dH[l], ld_h(), width, 1.0f, s));
    }
    HIPCHK(dalloc(&dY, (size_t)c * 2, false));
    HIPCHK(dalloc(&dDY, (size_t)c * 2, false));
    HIPCHK(dalloc(&dD0, (size_t)c * width, false));
    HIPCHK(dalloc(&dD1, (size_t)c * width, false));
    HIPCHK(dalloc(&dT, (size_t)c * 2, false));
    HIPCHK(dalloc(&dIdx, (size_t)c, false));
    HIPCHK(dalloc(&dLoss, 1));
    cap = c;
    return SPEC_OK;
}

namespace spec_host {

spec_status mlp_forward_x(spec_mlp_s* net, int rows, const float* X, int ldx, hipStream_t s) {
    const float* in = X;
    int ldin = ldx;
    for (int l = 0; l < net->nl; ++l) {
        const float* W = net->dP + net->off[l];
        const int K = net->dims[l] + 1, N = net->dims[l + 1];
        if (l < net->nl - 1) {
            HIPCHK(gemm_f32(false, false, net->bf16, GEMM_GELU, rows, N, K, in, ldin, W, N, net->dZ[l], net->width,
                            net->dH[l], net->ld_h(), s));
            in = net->dH[l];
            ldin = net->ld_h();
        } else {
            HIPCHK(gemm_f32(false, false, net->bf16, GEMM_STORE, rows, N, K, in, ldin, W, N, net->dY, 2, nullptr, 0,
                            s));
        }
    }
    return SPEC_OK;
}

spec_status mlp_backward(spec_mlp_s* net, int rows, const float* X, int ldx, float* g, hipStream_t s) {
    float* dcur = net->dDY;
    int ldcur = 2;
    for (int l = net->nl - 1; l >= 0; --l) {
        const float* in = l == 0 ? X : net->dH[l - 1];
        const int ldin = l == 0 ? ldx : net->ld_h();
        const int M = net->dims[l] + 1, N = net->dims[l + 1];
        // [dW_l; db_l] = [H_{l-1}, 1]^T delta_l
        HIPCHK(gemm_f32(true, false, net->bf16, GEMM_STORE, M, N, rows, in, ldin, dcur, ldcur, g + net->off[l], N,
                        nullptr, 0, s));
        if (l > 0) {
            // delta_{l-1} = (delta_l W_l^T) * GELU'(Z_{l-1})
            float* dnext = dcur == net->dD0 ? net->dD1 : net->dD0;
            HIPCHK(gemm_f32(false, true, net->bf16, GEMM_GELU_BWD, rows, net->dims[l], N, dcur, ldcur,
                            net->dP + net->off[l], N, dnext, net->width, net->dZ[l - 1], net->width, s));
            dcur = dnext;
            ldcur = net->width;
        }
    }
    return SPEC_OK;
}

spec_status mlp_predict_rows(spec_mlp_s* net, int rows, const double* x, int ldx, const double* v, int ldv,
                             hipStream_t s) {
    SPCHK(net->ensure(rows, s));
    HIPCHK(mlp_features(rows, net->n, net->nextra, x, ldx, v, ldv, net->dMu, net->dIsd, net->dX, net->ld_in(), s));
    return mlp_forward_x(net, rows, net->dX, net->ld_in(), s);
}

}  // namespace spec_host

namespace {

double quantile(std::vector<double> v, double q) {
    if (v.empty()) return NAN;
    const size_t k = std::min(v.size() - 1, (size_t)std::floor(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
}

}  // namespace

extern "C" {

spec_status spec_mlp_create(int n, int width, int hidden, int use_bf16, uint64_t seed, spec_mlp* out) {
    return spec_mlp_create_ex(n, width, hidden, use_bf16, seed, 0, out);
}

spec_status spec_mlp_create_ex(int n, int width, int hidden, int use_bf16, uint64_t seed, int products,
                               spec_mlp* out) {
    if (!out || n < 1 || width < 1 || width > 1024 || hidden < 1 || hidden > MLP_MAX_LAYERS - 1 || products < 0 ||
        products > 1)
        return SPEC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return SPEC_EDEVICE;
    spec_mlp_s* net = new spec_mlp_s();
    (void)hipGetDevice(&net->device);
    net->n = n;
    net->width = width;
    net->hidden = hidden;
    net->nl = hidden + 1;
    net->bf16 = use_bf16 ? 1 : 0;
    net->nextra = products ? 2 : 0;
    net->dims[0] = 2 * n + net->nextra;
    for (int l = 1; l <= hidden; ++l) net->dims[l] = width;
    net->dims[hidden + 1] = 2;
    int64_t o = 0;
    for (int l = 0; l < net->nl; ++l) {
        net->off[l] = o;
        o += (int64_t)(net->dims[l] + 1) * net->dims[l + 1];
    }
    net->np = o;
    hipError_t e = dalloc(&net->dP, (size_t)o, false);
    if (e == hipSuccess) e = dalloc(&net->dG, (size_t)o);
    if (e == hipSuccess) e = dalloc(&net->dM, (size_t)o);
    if (e == hipSuccess) e = dalloc(&net->dV, (size_t)o);
    const int nin = net->dims[0];
    if (e == hipSuccess) e = dalloc(&net->dMu, (size_t)nin);
    std::vector<float> ones((size_t)nin, 1.0f);
    if (e == hipSuccess) e = dalloc(&net->dIsd, (size_t)nin, false);
    if (e == hipSuccess) e = hipMemcpy(net->dIsd, ones.data(), sizeof(float) * ones.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = mlp_init(net->nl, net->dims, net->dP, seed, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        spec_mlp_destroy(net);
        return from_hip(e);
    }
    *out = net;
    return SPEC_OK;
}

spec_status spec_mlp_destroy(spec_mlp net) {
    if (!net) return SPEC_EINVAL;
    (void)hipDeviceSynchronize();
    net->free_work();
    dfree(net->dP); dfree(net->dG); dfree(net->dM); dfree(net->dV); dfree(net->dMu); dfree(net->dIsd);
    delete net;
    return SPEC_OK;
}

spec_status spec_mlp_standardization(spec_mlp net, float* mu, float* isd, float* target) {
    if (!net || !mu || !isd || !target) return SPEC_EINVAL;
    HIPCHK(hipMemcpy(mu, net->dMu, sizeof(float) * net->dims[0], hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(isd, net->dIsd, sizeof(float) * net->dims[0], hipMemcpyDeviceToHost));
    target[0] = net->tmu[0];
    target[1] = net->tmu[1];
    target[2] = net->tsd[0];
    target[3] = net->tsd[1];
    return SPEC_OK;
}

spec_status spec_mlp_nparams(spec_mlp net, long long* np) {
    if (!net || !np) return SPEC_EINVAL;
    *np = net->np;
    return SPEC_OK;
}

spec_status spec_mlp_get_params(spec_mlp net, float* host) {
    if (!net || !host) return SPEC_EINVAL;
    HIPCHK(hipMemcpy(host, net->dP, sizeof(float) * net->np, hipMemcpyDeviceToHost));
    return SPEC_OK;
}

spec_status spec_mlp_set_params(spec_mlp net, const float* host) {
    if (!net || !host) return SPEC_EINVAL;
    HIPCHK(hipMemcpy(net->dP, host, sizeof(float) * net->np, hipMemcpyHostToDevice));
    return SPEC_OK;
}

spec_status spec_mlp_forward_dev(spec_mlp net, int rows, const float* X, float* Y, void* stream) {
    if (!net || rows < 0 || (rows && (!X || !Y))) return SPEC_EINVAL;
    if (rows == 0) return SPEC_OK;
    hipStream_t s = (hipStream_t)stream;
    SPCHK(net->ensure(rows, s));
    HIPCHK(mlp_augment(rows, net->dims[0], X, net->dims[0], net->dX, net->ld_in(), s));
    SPCHK(mlp_forward_x(net, rows, net->dX, net->ld_in(), s));
    HIPCHK(hipMemcpyAsync(Y, net->dY, sizeof(float) * rows * 2, hipMemcpyDeviceToDevice, s));
    return SPEC_OK;
}

spec_status spec_mlp_loss_grad_dev(spec_mlp net, int rows, const float* X, const float* T, float* grad,
                                   double* loss, void* stream) {
    if (!net || rows < 1 || !X || !T || !grad) return SPEC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    SPCHK(net->ensure(rows, s));
    HIPCHK(mlp_augment(rows, net->dims[0], X, net->dims[0], net->dX, net->ld_in(), s));
    SPCHK(mlp_forward_x(net, rows, net->dX, net->ld_in(), s));
    HIPCHK(hipMemsetAsync(net->dLoss, 0, sizeof(double), s));
    HIPCHK(mlp_mse(rows, 2, net->dY, 2, T, net->dDY, net->dLoss, s));
    SPCHK(mlp_backward(net, rows, net->dX, net->ld_in(), grad, s));
    double l = 0.0;
    HIPCHK(hipMemcpyAsync(&l, net->dLoss, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (loss) *loss = l / (2.0 * rows);
    return SPEC_OK;
}

spec_status spec_mlp_adam_dev(spec_mlp net, const float* grad, double lr, void* stream) {
    if (!net || !grad || !(lr > 0.0)) return SPEC_EINVAL;
    net->step += 1;
    HIPCHK(mlp_adam(net->np, net->dP, grad, net->dM, net->dV, net->step, (float)lr, 0.9f, 0.999f, 1e-8f,
                    (hipStream_t)stream));
    return SPEC_OK;
}

spec_status spec_mlp_train_dev(spec_mlp net, int rows, const double* x, const double* v, const double* t_minus,
                               const double* t_plus, const spec_mlp_train_params* p, spec_mlp_train_stats* st,
                               void* stream) {
    if (!net || !p || rows < 2 || !x || !v || !t_minus || !t_plus) return SPEC_EINVAL;
    const int epochs = p->epochs > 0 ? p->epochs : 20;
    const int batch = p->batch > 0 ? p->batch : 4096;
    const double lr0 = p->lr > 0.0 ? p->lr : 1e-3;
    const double lr1 = p->lr_final > 0.0 ? p->lr_final : 1e-5;
    const double vf = p->val_frac > 0.0 && p->val_frac < 1.0 ? p->val_frac : 0.1;
    const double qq = p->quantile > 0.0 && p->quantile < 1.0 ? p->quantile : 0.999;
    const int nval = std::max(1, (int)std::lround(vf * rows));
    const int ntrain = rows - nval;
    if (ntrain < 1) return SPEC_EINVAL;
    const int n = net->n, nin = net->dims[0];
    hipStream_t s = (hipStream_t)stream;

    // targets on the host (rows x 2 doubles): standardisation of the training rows
    std::vector<double> hm(rows), hp(rows);
    HIPCHK(hipMemcpyAsync(hm.data(), t_minus, sizeof(double) * rows, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hp.data(), t_plus, sizeof(double) * rows, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int r = 0; r < rows; ++r)
        if (!(hp[r] > 0.0) || !std::isfinite(hp[r]) || !(hm[r] < 0.0) || !std::isfinite(hm[r])) return SPEC_EINVAL;
    double s0 = 0, q0 = 0, s1 = 0, q1 = 0;
    for (int r = 0; r < ntrain; ++r) {
        const double a = std::log(hp[r]), b = std::log(-hm[r]);
        s0 += a; q0 += a * a; s1 += b; q1 += b * b;
    }
    const double m0 = s0 / ntrain, m1 = s1 / ntrain;
    const double sd0 = std::sqrt(std::max(q0 / ntrain - m0 * m0, 1e-12));
    const double sd1 = std::sqrt(std::max(q1 / ntrain - m1 * m1, 1e-12));
    net->tmu[0] = (float)m0; net->tsd[0] = (float)sd0;
    net->tmu[1] = (float)m1; net->tsd[1] = (float)sd1;

    // feature standardisation from the training rows
    double *dSum = nullptr, *dSq = nullptr;
    HIPCHK(dalloc(&dSum, (size_t)nin));
    HIPCHK(dalloc(&dSq, (size_t)nin));
    HIPCHK(mlp_col_moments(ntrain, n, x, n, dSum, dSq, s));
    HIPCHK(mlp_col_moments(ntrain, n, v, n, dSum + n, dSq + n, s));
    if (net->nextra) {
        double* dPr = nullptr;
        HIPCHK(dalloc(&dPr, (size_t)2 * ntrain, false));
        HIPCHK(mlp_products(ntrain, n, x, n, v, n, dPr, s));
        HIPCHK(mlp_col_moments(ntrain, 2, dPr, 2, dSum + 2 * n, dSq + 2 * n, s));
        HIPCHK(hipStreamSynchronize(s));
        dfree(dPr);
    }
    std::vector<double> hs(nin), hq(nin);
    HIPCHK(hipMemcpyAsync(hs.data(), dSum, sizeof(double) * nin, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hq.data(), dSq, sizeof(double) * nin, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dfree(dSum);
    dfree(dSq);
    std::vector<float> mu(nin), isd(nin);
    for (int i = 0; i < nin; ++i) {
        const double mm = hs[i] / ntrain;
        const double var = std::max(hq[i] / ntrain - mm * mm, 1e-24);
        mu[i] = (float)mm;
        isd[i] = (float)(1.0 / std::sqrt(var));
    }
    HIPCHK(hipMemcpy(net->dMu, mu.data(), sizeof(float) * nin, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(net->dIsd, isd.data(), sizeof(float) * nin, hipMemcpyHostToDevice));

    // all features (rows x ld_in) and standardised targets (rows x 2) in FP32
    const int ldx = net->ld_in();
    float *dXall = nullptr, *dTall = nullptr, *dTm = nullptr;
    HIPCHK(dalloc(&dXall, (size_t)rows * ldx, false));
    HIPCHK(dalloc(&dTall, (size_t)rows * 2, false));
    HIPCHK(dalloc(&dTm, (size_t)4, false));
    const float tmi[4] = {net->tmu[0], net->tmu[1], 1.0f / net->tsd[0], 1.0f / net->tsd[1]};
    HIPCHK(hipMemcpy(dTm, tmi, sizeof(tmi), hipMemcpyHostToDevice));
    HIPCHK(mlp_features(rows, n, net->nextra, x, n, v, n, net->dMu, net->dIsd, dXall, ldx, s));
    HIPCHK(mlp_targets(rows, t_minus, t_plus, dTm, dTm + 2, dTall, s));

    const int cap_rows = std::max(batch, std::min(nval, 65536));
    SPCHK(net->ensure(cap_rows, s));
    const long long steps = std::max(1LL, (long long)epochs * ntrain / batch);
    const long long per_epoch = std::max(1LL, (long long)ntrain / batch);
    const double pi = 3.14159265358979323846;
    double train_loss = 0.0;
    // early stopping: the validation loss after every epoch, the best parameters kept
    const bool keep_best = p->keep_best != 0;
    float* dBest = nullptr;
    double* dVl = nullptr;
    double best_vl = INFINITY;
    int best_epoch = epochs;
    if (keep_best) {
        HIPCHK(dalloc(&dBest, (size_t)net->np, false));
        HIPCHK(dalloc(&dVl, (size_t)1));
    }
    auto val_loss_now = [&](double* out) -> spec_status {
        HIPCHK(hipMemsetAsync(dVl, 0, sizeof(double), s));
        for (int r0 = 0; r0 < nval; r0 += cap_rows) {
            const int cnt = std::min(cap_rows, nval - r0);
            SPCHK(mlp_forward_x(net, cnt, dXall + (size_t)(ntrain + r0) * ldx, ldx, s));
            HIPCHK(mlp_mse(cnt, 2, net->dY, 2, dTall + (size_t)(ntrain + r0) * 2, net->dDY, dVl, s));
        }
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, dVl, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *out = v / (2.0 * nval);
        return SPEC_OK;
    };
    for (long long it = 0; it < steps; ++it) {
        const double lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + std::cos(pi * (double)it / (double)steps));
        if (it == steps - per_epoch || (it == 0 && steps <= per_epoch))
            HIPCHK(hipMemsetAsync(net->dLoss, 0, sizeof(double), s));
        HIPCHK(mlp_sample_rows(batch, ntrain, p->seed, (uint32_t)it, net->dIdx, s));
        HIPCHK(mlp_gather(batch, ldx, net->dIdx, dXall, ldx, net->dX, ldx, s));
        HIPCHK(mlp_gather(batch, 2, net->dIdx, dTall, 2, net->dT, 2, s));
        SPCHK(mlp_forward_x(net, batch, net->dX, ldx, s));
        HIPCHK(mlp_mse(batch, 2, net->dY, 2, net->dT, net->dDY, net->dLoss, s));
        SPCHK(mlp_backward(net, batch, net->dX, ldx, net->dG, s));
        net->step += 1;
        HIPCHK(mlp_adam(net->np, net->dP, net->dG, net->dM, net->dV, net->step, (float)lr, 0.9f, 0.999f, 1e-8f, s));
        if (keep_best && ((it + 1) % per_epoch == 0 || it + 1 == steps)) {
            double vl = 0.0;
            SPCHK(val_loss_now(&vl));
            if (vl < best_vl) {
                best_vl = vl;
                best_epoch = (int)std::min<long long>(epochs, (it + 1 + per_epoch - 1) / per_epoch);
                HIPCHK(hipMemcpyAsync(dBest, net->dP, sizeof(float) * net->np, hipMemcpyDeviceToDevice, s));
            }
        }
    }
    if (keep_best) {
        HIPCHK(hipMemcpyAsync(net->dP, dBest, sizeof(float) * net->np, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        dfree(dBest);
        dfree(dVl);
    }
    {
        double l = 0.0;
        HIPCHK(hipMemcpyAsync(&l, net->dLoss, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const long long counted = std::min(steps, per_epoch);
        train_loss = l / (2.0 * batch * counted);
    }

    // validation rows: errors of log t+ and the loss
    std::vector<float> yv((size_t)nval * 2);
    for (int r0 = 0; r0 < nval; r0 += cap_rows) {
        const int cnt = std::min(cap_rows, nval - r0);
        SPCHK(mlp_forward_x(net, cnt, dXall + (size_t)(ntrain + r0) * ldx, ldx, s));
        HIPCHK(hipMemcpyAsync(yv.data() + (size_t)r0 * 2, net->dY, sizeof(float) * cnt * 2, hipMemcpyDeviceToHost,
                              s));
    }
    std::vector<float> tv((size_t)nval * 2);
    HIPCHK(hipMemcpyAsync(tv.data(), dTall + (size_t)ntrain * 2, sizeof(float) * nval * 2, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dfree(dXall);
    dfree(dTall);
    dfree(dTm);
    std::vector<double> err(nval);
    double vl = 0.0, vc = 0.0;
    for (int r = 0; r < nval; ++r) {
        const double d0 = (double)yv[2 * r] - tv[2 * r], d1 = (double)yv[2 * r + 1] - tv[2 * r + 1];
        vl += d0 * d0 + d1 * d1;
        vc += (double)tv[2 * r] * tv[2 * r] + (double)tv[2 * r + 1] * tv[2 * r + 1];
        const double pred = (double)yv[2 * r] * net->tsd[0] + net->tmu[0];
        err[r] = std::fabs(pred - std::log(hp[ntrain + r]));
    }
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->train_loss = train_loss;
        st->val_loss = vl / (2.0 * nval);
        st->val_loss_const = vc / (2.0 * nval);
        st->best_epoch = best_epoch;
        st->delta = quantile(err, qq);
        st->err_median = quantile(err, 0.5);
        st->err_p99 = quantile(err, 0.99);
        st->err_max = *std::max_element(err.begin(), err.end());
        st->steps = (double)steps;
        st->val_rows = nval;
        const double lv[8] = {0.5, 0.7, 0.8, 0.9, 0.95, 0.99, 0.995, 0.999};
        for (int i = 0; i < 8; ++i) st->err_q[i] = quantile(err, lv[i]);
    }
    return SPEC_OK;
}

spec_status spec_mlp_train(spec_mlp net, int rows, const double* x, const double* v, const double* t_minus,
                           const double* t_plus, const spec_mlp_train_params* p, spec_mlp_train_stats* st) {
    if (!net || !p || rows < 2 || !x || !v || !t_minus || !t_plus) return SPEC_EINVAL;
    const size_t rn = (size_t)rows * net->n;
    double *dx = nullptr, *dv = nullptr, *dm = nullptr, *dp = nullptr;
    spec_status rc = SPEC_OK;
    hipError_t e = dalloc(&dx, rn, false);
    if (e == hipSuccess) e = dalloc(&dv, rn, false);
    if (e == hipSuccess) e = dalloc(&dm, (size_t)rows, false);
    if (e == hipSuccess) e = dalloc(&dp, (size_t)rows, false);
    if (e == hipSuccess) e = hipMemcpy(dx, x, sizeof(double) * rn, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dv, v, sizeof(double) * rn, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dm, t_minus, sizeof(double) * rows, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dp, t_plus, sizeof(double) * rows, hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = from_hip(e);
    if (rc == SPEC_OK) rc = spec_mlp_train_dev(net, rows, dx, dv, dm, dp, p, st, nullptr);
    dfree(dx);
    dfree(dv);
    dfree(dm);
    dfree(dp);
    return rc;
}

spec_status spec_mlp_predict_dev(spec_mlp net, int rows, const double* x, const double* v, double* log_tp,
                                 double* log_neg_tm, void* stream) {
    if (!net || rows < 0 || (rows && (!x || !v))) return SPEC_EINVAL;
    if (rows == 0) return SPEC_OK;
    hipStream_t s = (hipStream_t)stream;
    for (int r0 = 0; r0 < rows; r0 += 65536) {
        const int cnt = std::min(65536, rows - r0);
        SPCHK(mlp_predict_rows(net, cnt, x + (size_t)r0 * net->n, net->n, v + (size_t)r0 * net->n, net->n, s));
        HIPCHK(mlp_unstandardise(cnt, net->dY, 2, net->tmu[0], net->tsd[0], net->tmu[1], net->tsd[1],
                                 log_tp ? log_tp + r0 : nullptr, log_neg_tm ? log_neg_tm + r0 : nullptr, s));
    }
    return SPEC_OK;
}

// ------------------------------------------------------------ diagnostics

spec_status spec_diag_mfma_raw(int kind, int trials, const float* a, const float* b, float* d) {
    if ((kind != 0 && kind != 1) || trials < 1 || !a || !b || !d) return SPEC_EINVAL;
    const size_t per = kind == 0 ? 64 : 512;
    float *da = nullptr, *db = nullptr, *dd = nullptr;
    hipError_t e = dalloc(&da, per * trials, false);
    if (e == hipSuccess) e = dalloc(&db, per * trials, false);
    if (e == hipSuccess) e = dalloc(&dd, (size_t)256 * trials, false);
    if (e == hipSuccess) e = hipMemcpy(da, a, sizeof(float) * per * trials, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(db, b, sizeof(float) * per * trials, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = mfma_raw_probe(kind, trials, da, db, dd, nullptr);
    if (e == hipSuccess) e = hipMemcpy(d, dd, sizeof(float) * 256 * trials, hipMemcpyDeviceToHost);
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dd);
    return from_hip(e);
}

spec_status spec_diag_gemm_f32(int ta, int tb, int bf16, int mode, int M, int N, int K, const float* A, int lda,
                               const float* B, int ldb, float* C, int ldc, float* aux, int ldaux) {
    if (M < 1 || N < 1 || K < 1 || !A || !B || !C || mode < 0 || mode > 2 || (mode && !aux)) return SPEC_EINVAL;
    const size_t na = ta ? (size_t)K * lda : (size_t)M * lda;
    const size_t nb = tb ? (size_t)N * ldb : (size_t)K * ldb;
    const size_t nc = (size_t)M * ldc, nx = mode ? (size_t)M * ldaux : 0;
    if ((ta ? lda < M : lda < K) || (tb ? ldb < K : ldb < N) || ldc < N || (mode && ldaux < N)) return SPEC_EINVAL;
    float *dA = nullptr, *dB = nullptr, *dC = nullptr, *dX = nullptr;
    hipError_t e = dalloc(&dA, na, false);
    if (e == hipSuccess) e = dalloc(&dB, nb, false);
    if (e == hipSuccess) e = dalloc(&dC, nc, false);
    if (e == hipSuccess && nx) e = dalloc(&dX, nx, false);
    if (e == hipSuccess) e = hipMemcpy(dA, A, sizeof(float) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dB, B, sizeof(float) * nb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dC, C, sizeof(float) * nc, hipMemcpyHostToDevice);
    if (e == hipSuccess && nx) e = hipMemcpy(dX, aux, sizeof(float) * nx, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = gemm_f32(ta != 0, tb != 0, bf16 != 0, mode, M, N, K, dA, lda, dB, ldb, dC, ldc, dX, ldaux, nullptr);
    if (e == hipSuccess) e = hipMemcpy(C, dC, sizeof(float) * nc, hipMemcpyDeviceToHost);
    if (e == hipSuccess && nx) e = hipMemcpy(aux, dX, sizeof(float) * nx, hipMemcpyDeviceToHost);
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dC);
    (void)hipFree(dX);
    return from_hip(e);
}

}  // extern "C"
