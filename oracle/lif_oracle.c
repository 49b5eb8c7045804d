/*
 * CPU oracle for the homogeneous (matrix-form, "MAT") leaky integrate-and-fire
 * simulation with synaptic delays of SuperNeuro (Date et al., ICONS'23, §2.1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the GPU path is checked against.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header or table with the HIP library; the product never calls it.
 *
 * Arithmetic is IEEE double.  The workloads use dyadic values (multiples of
 * 2^-6) whose every partial sum stays far below 2^17, so every sum below is
 * exact in double and in float alike, in any order.  With check_exact != 0 the
 * oracle verifies that premise step by step and returns OR_NONEXACT when it
 * fails (the computed result is still written out).
 *
 * Model, per trial b, neuron j, step t = 0 .. T-1 (state of step -1: V = r,
 * refractory counter 0, no spikes):
 *   1. constant leak towards the reset state r (§2.1, leak paragraph): above r
 *      subtract lambda, below r add lambda, never crossing r;
 *   2. add the spikes of earlier steps through the weight matrix, a synapse
 *      i->j of weight w and integer delay d >= 1 delivering w at t when i
 *      spiked at t-d (§2.1: W row = pre, column = post; delay d realised in
 *      the paper by a chain of d-1 unit-delay proxy neurons);
 *   3. add the external spikes of step t, scaled by the amplitude a_j;
 *   4. spike candidate c = (U > threshold)  (strict: the ABM description in
 *      §2.2 states "greater than", and the leak notion is shared);
 *   5. refractory period: a neuron whose counter is non-zero has its spike
 *      zeroed and its counter decremented (§2.1, last step);
 *   6. an emitted spike resets the state to r and starts a refractory window
 *      of R steps (reset state and refractory period are the neuron
 *      parameters listed in §2.1).
 * A suppressed (refractory) super-threshold neuron keeps U: only its spike is
 * removed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_NONEXACT (-6)

/* 2^17: bound on |partial sum| that keeps multiples of 2^-6 exact in binary32
 * (2^17 / 2^-6 = 2^23 < 2^24). */
static const double EXACT_LIMIT = 131072.0;

/* Is x a finite multiple of 2^-6 below the exactness limit? */
static int on_grid(double x) {
    if (!isfinite(x) || fabs(x) >= EXACT_LIMIT) return 0;
    double s = x * 64.0;
    return s == floor(s);
}

/* Step 1: constant leak towards r, never crossing it (§2.1). */
static double apply_leak(double v, double r, double lambda) {
    if (v > r) {
        double u = v - lambda;
        return u < r ? r : u;
    }
    if (v < r) {
        double u = v + lambda;
        return u > r ? r : u;
    }
    return v;
}

/* Steps 4-6 for one neuron; returns the emitted spike (0/1) and updates
 * *v (new state) and *ref (remaining refractory steps). */
static int fire_and_reset(double u, double theta, double r, int32_t R,
                          double* v, int32_t* ref) {
    int candidate = u > theta;                /* step 4 */
    int spike;
    if (*ref > 0) {                           /* step 5 */
        spike = 0;
        *ref = *ref - 1;
    } else {
        spike = candidate;
    }
    if (spike) {                              /* step 6 */
        *v = r;
        *ref = R;
    } else {
        *v = u;
    }
    return spike;
}

static int check_params(int32_t N, const double* theta, const double* leak,
                        const double* reset, const int32_t* refractory,
                        const double* amplitude) {
    for (int32_t j = 0; j < N; ++j) {
        if (!on_grid(theta[j]) || !on_grid(reset[j]) || !on_grid(amplitude[j]))
            return 0;
        if (!(leak[j] >= 0.0)) return 0;
        if (!isinf(leak[j]) && !on_grid(leak[j])) return 0;
        if (refractory[j] < 0) return 0;
    }
    return 1;
}

/*
 * Sparse synapse list (COO: pre[k] -> post[k], weight w[k], delay delay[k]).
 * ext and spikes are byte arrays [B][T][N] holding 0 or 1.
 * V_out [B][N] and ref_out [B][N] receive the state after step T-1.
 */
static int lif_sparse(int32_t N, int32_t B, int32_t D, int32_t T,
                      const double* theta, const double* leak, const double* reset,
                      const int32_t* refractory, const double* amplitude,
                      int64_t nnz, const int32_t* pre, const int32_t* post,
                      const double* w, const int32_t* delay,
                      const uint8_t* history, const uint8_t* ext, uint8_t* spikes,
                      double* V_out, int32_t* ref_out, int check_exact);

int or_lif_sparse(int32_t N, int32_t B, int32_t D, int32_t T,
                  const double* theta, const double* leak, const double* reset,
                  const int32_t* refractory, const double* amplitude,
                  int64_t nnz, const int32_t* pre, const int32_t* post,
                  const double* w, const int32_t* delay,
                  const uint8_t* ext, uint8_t* spikes,
                  double* V_out, int32_t* ref_out, int check_exact) {
    return lif_sparse(N, B, D, T, theta, leak, reset, refractory, amplitude, nnz, pre, post, w, delay,
                      NULL, ext, spikes, V_out, ref_out, check_exact);
}

/*
 * The same update driven by a given spike history: step 2 takes the source
 * spikes s_pre(t - d) from history [B][T][N] instead of the spikes computed
 * here.  Fed the network's own raster it reproduces that raster and the final
 * state; given only the synapses into some post-neurons, it reproduces those
 * neurons' columns, so a large net can be checked in independent post ranges
 * (every range checked = the whole raster, by induction over t).
 */
int or_lif_sparse_driven(int32_t N, int32_t B, int32_t D, int32_t T,
                         const double* theta, const double* leak, const double* reset,
                         const int32_t* refractory, const double* amplitude,
                         int64_t nnz, const int32_t* pre, const int32_t* post,
                         const double* w, const int32_t* delay,
                         const uint8_t* history, const uint8_t* ext, uint8_t* spikes,
                         double* V_out, int32_t* ref_out, int check_exact) {
    if (!history) return OR_EINVAL;
    return lif_sparse(N, B, D, T, theta, leak, reset, refractory, amplitude, nnz, pre, post, w, delay,
                      history, ext, spikes, V_out, ref_out, check_exact);
}

static int lif_sparse(int32_t N, int32_t B, int32_t D, int32_t T,
                      const double* theta, const double* leak, const double* reset,
                      const int32_t* refractory, const double* amplitude,
                      int64_t nnz, const int32_t* pre, const int32_t* post,
                      const double* w, const int32_t* delay,
                      const uint8_t* history, const uint8_t* ext, uint8_t* spikes,
                      double* V_out, int32_t* ref_out, int check_exact) {
    if (N < 1 || B < 1 || D < 1 || T < 0 || nnz < 0) return OR_EINVAL;
    for (int64_t k = 0; k < nnz; ++k) {
        if (pre[k] < 0 || pre[k] >= N || post[k] < 0 || post[k] >= N) return OR_EINVAL;
        if (delay[k] < 1 || delay[k] > D) return OR_EINVAL;
        if (!isfinite(w[k])) return OR_EINVAL;
    }
    int exact = 1;
    if (check_exact) {
        if (!check_params(N, theta, leak, reset, refractory, amplitude)) exact = 0;
        for (int64_t k = 0; k < nnz; ++k)
            if (!on_grid(w[k])) exact = 0;
    }
    /* in_abs[j] = sum of |w| over synapses into j: bounds the synaptic term. */
    double* in_abs = (double*)calloc((size_t)N, sizeof(double));
    double* U = (double*)malloc((size_t)N * sizeof(double));
    if (!in_abs || !U) { free(in_abs); free(U); return OR_ENOMEM; }
    for (int64_t k = 0; k < nnz; ++k) in_abs[post[k]] += fabs(w[k]);

    for (int32_t b = 0; b < B; ++b) {
        double* V = V_out + (size_t)b * N;
        int32_t* ref = ref_out + (size_t)b * N;
        const uint8_t* xb = ext + (size_t)b * T * N;
        uint8_t* sb = spikes + (size_t)b * T * N;
        /* source spikes: the given history, else the spikes computed here */
        const uint8_t* src = history ? history + (size_t)b * T * N : sb;
        for (int32_t j = 0; j < N; ++j) { V[j] = reset[j]; ref[j] = 0; }

        for (int32_t t = 0; t < T; ++t) {
            /* 1. leak */
            for (int32_t j = 0; j < N; ++j) {
                U[j] = apply_leak(V[j], reset[j], leak[j]);
                if (check_exact && !(fabs(U[j]) + in_abs[j] + fabs(amplitude[j]) < EXACT_LIMIT))
                    exact = 0;
            }
            /* 2. delayed synaptic input: w * s_pre(t - d) */
            for (int64_t k = 0; k < nnz; ++k) {
                int32_t src_t = t - delay[k];
                if (src_t < 0) continue;
                if (src[(size_t)src_t * N + pre[k]]) U[post[k]] += w[k];
            }
            /* 3. external spikes */
            for (int32_t j = 0; j < N; ++j)
                if (xb[(size_t)t * N + j]) U[j] += amplitude[j];
            /* 4-6. threshold, refractory, reset */
            for (int32_t j = 0; j < N; ++j)
                sb[(size_t)t * N + j] =
                    (uint8_t)fire_and_reset(U[j], theta[j], reset[j], refractory[j], &V[j], &ref[j]);
        }
    }
    free(in_abs);
    free(U);
    return exact ? OR_OK : OR_NONEXACT;
}

/*
 * Spike-timing-dependent plasticity on the synapse list.  §2.1 names STDP as
 * the learning of the matrix mode but gives no rule, window or constants, so
 * the rule below is a chosen one (parity of the rule itself is unpinned by the
 * paper); it keeps every weight on the 2^-6 grid when the tables are on it.
 * One trial.  A spike of pre-neuron i at step tau arrives at post-neuron j at
 * t_a = tau + d.  After the update of step t (the new weights act from step
 * t + 1), for every synapse i->j of delay d:
 *   - potentiation, if j spikes at t: the latest arrival t_a <= t with
 *     t - t_a < W adds ltp[t - t_a];
 *   - depression, if a spike of i arrives at t (i spiked at t - d): the latest
 *     spike of j at t_post < t with t - t_post <= W subtracts ltd[t - t_post - 1];
 *   - then w = min(max(w, w_min), w_max).
 * Each synapse's change depends on spike times only, so the order in which
 * synapses are visited does not matter.  w is updated in place.
 */
int or_lif_stdp(int32_t N, int32_t D, int32_t T,
                const double* theta, const double* leak, const double* reset,
                const int32_t* refractory, const double* amplitude,
                int64_t nnz, const int32_t* pre, const int32_t* post,
                double* w, const int32_t* delay,
                const uint8_t* ext, uint8_t* spikes,
                double* V, int32_t* ref, int32_t W, const double* ltp, const double* ltd,
                double w_min, double w_max, int check_exact) {
    if (N < 1 || D < 1 || T < 0 || nnz < 0 || W < 1 || W > 16 || !(w_min <= w_max)) return OR_EINVAL;
    for (int64_t k = 0; k < nnz; ++k) {
        if (pre[k] < 0 || pre[k] >= N || post[k] < 0 || post[k] >= N) return OR_EINVAL;
        if (delay[k] < 1 || delay[k] > D) return OR_EINVAL;
        if (!isfinite(w[k])) return OR_EINVAL;
    }
    int exact = 1;
    if (check_exact) {
        if (!check_params(N, theta, leak, reset, refractory, amplitude)) exact = 0;
        for (int64_t k = 0; k < nnz; ++k)
            if (!on_grid(w[k])) exact = 0;
        for (int32_t k = 0; k < W; ++k)
            if (!on_grid(ltp[k]) || !on_grid(ltd[k])) exact = 0;
        if (!on_grid(w_min) || !on_grid(w_max)) exact = 0;
    }
    double* in_abs = (double*)malloc((size_t)N * sizeof(double));
    double* U = (double*)malloc((size_t)N * sizeof(double));
    if (!in_abs || !U) { free(in_abs); free(U); return OR_ENOMEM; }
    for (int32_t j = 0; j < N; ++j) { V[j] = reset[j]; ref[j] = 0; }

    for (int32_t t = 0; t < T; ++t) {
        for (int32_t j = 0; j < N; ++j) in_abs[j] = 0.0;
        for (int64_t k = 0; k < nnz; ++k) in_abs[post[k]] += fabs(w[k]);
        /* steps 1-6 of the model, as in or_lif_sparse */
        for (int32_t j = 0; j < N; ++j) {
            U[j] = apply_leak(V[j], reset[j], leak[j]);
            if (check_exact && !(fabs(U[j]) + in_abs[j] + fabs(amplitude[j]) < EXACT_LIMIT)) exact = 0;
        }
        for (int64_t k = 0; k < nnz; ++k) {
            int32_t src_t = t - delay[k];
            if (src_t >= 0 && spikes[(size_t)src_t * N + pre[k]]) U[post[k]] += w[k];
        }
        for (int32_t j = 0; j < N; ++j)
            if (ext[(size_t)t * N + j]) U[j] += amplitude[j];
        for (int32_t j = 0; j < N; ++j)
            spikes[(size_t)t * N + j] =
                (uint8_t)fire_and_reset(U[j], theta[j], reset[j], refractory[j], &V[j], &ref[j]);
        /* plasticity from the spike times up to and including t */
        for (int64_t k = 0; k < nnz; ++k) {
            const int32_t i = pre[k], j = post[k], d = delay[k];
            double change = 0.0;
            if (spikes[(size_t)t * N + j]) {
                for (int32_t lag = 0; lag < W; ++lag) {   /* arrival at t - lag */
                    int32_t tau = t - lag - d;
                    if (tau < 0) break;
                    if (spikes[(size_t)tau * N + i]) { change += ltp[lag]; break; }
                }
            }
            if (t - d >= 0 && spikes[(size_t)(t - d) * N + i]) {
                for (int32_t lag = 1; lag <= W; ++lag) {  /* post spike at t - lag */
                    if (t - lag < 0) break;
                    if (spikes[(size_t)(t - lag) * N + j]) { change -= ltd[lag - 1]; break; }
                }
            }
            if (change != 0.0 || w[k] < w_min || w[k] > w_max) {
                double x = w[k] + change;
                w[k] = x < w_min ? w_min : (x > w_max ? w_max : x);
            }
        }
    }
    free(in_abs);
    free(U);
    return exact ? OR_OK : OR_NONEXACT;
}

/*
 * Selected post-neurons of a dense delay-1 net, one at a time, given the
 * spike history of the whole network: for neuron j = posts[k] the update of
 * §2.1 over T steps, whose synaptic input at step t is the sum of W[i][j]
 * over the neurons i with history[b][t-1][i] = 1.  wcol [S][N] holds the
 * columns, wcol[k][i] = W[i][posts[k]]; parameter vectors and ext [B][T][N]
 * cover all N neurons.  Outputs: spikes [B][T][S], V_out and ref_out [B][S].
 * When `history` is the network's own raster, the outputs are that raster's
 * columns and the final state of the listed neurons, so a large net can be
 * checked neuron by neuron without simulating all of it.
 */
int or_lif_columns(int32_t N, int32_t B, int32_t T, int32_t S, const int32_t* posts,
                   const double* theta, const double* leak, const double* reset,
                   const int32_t* refractory, const double* amplitude,
                   const double* wcol, const uint8_t* history, const uint8_t* ext,
                   uint8_t* spikes, double* V_out, int32_t* ref_out, int check_exact) {
    if (N < 1 || B < 1 || T < 0 || S < 0) return OR_EINVAL;
    for (int32_t k = 0; k < S; ++k)
        if (posts[k] < 0 || posts[k] >= N) return OR_EINVAL;
    int exact = 1;
    if (check_exact && !check_params(N, theta, leak, reset, refractory, amplitude)) exact = 0;
    /* the neurons that spiked at every step, in ascending order, so the sum
     * over them visits the same terms as a scan of the whole history row */
    size_t total = 0;
    for (size_t q = 0; q < (size_t)B * T * N; ++q) total += history[q] != 0;
    int32_t* list = (int32_t*)malloc((total + 1) * sizeof(int32_t));
    size_t* first = (size_t*)malloc(((size_t)B * T + 1) * sizeof(size_t));
    if (!list || !first) { free(list); free(first); return OR_ENOMEM; }
    total = 0;
    for (size_t bt = 0; bt < (size_t)B * T; ++bt) {
        first[bt] = total;
        for (int32_t i = 0; i < N; ++i)
            if (history[bt * N + i]) list[total++] = i;
    }
    first[(size_t)B * T] = total;
    for (int32_t k = 0; k < S; ++k) {
        const int32_t j = posts[k];
        const double* w = wcol + (size_t)k * N;
        double in_abs = 0.0;
        for (int32_t i = 0; i < N; ++i) {
            if (!isfinite(w[i])) { free(list); free(first); return OR_EINVAL; }
            if (check_exact && w[i] != 0.0 && !on_grid(w[i])) exact = 0;
            in_abs += fabs(w[i]);
        }
        for (int32_t b = 0; b < B; ++b) {
            const uint8_t* xb = ext + (size_t)b * T * N;
            double V = reset[j];
            int32_t ref = 0;
            for (int32_t t = 0; t < T; ++t) {
                double U = apply_leak(V, reset[j], leak[j]);
                if (check_exact && !(fabs(U) + in_abs + fabs(amplitude[j]) < EXACT_LIMIT)) exact = 0;
                if (t > 0) {  /* neurons that spiked at t - 1 */
                    const size_t bt = (size_t)b * T + (t - 1);
                    for (size_t q = first[bt]; q < first[bt + 1]; ++q) U += w[list[q]];
                }
                if (xb[(size_t)t * N + j]) U += amplitude[j];
                spikes[((size_t)b * T + t) * S + k] =
                    (uint8_t)fire_and_reset(U, theta[j], reset[j], refractory[j], &V, &ref);
            }
            V_out[(size_t)b * S + k] = V;
            ref_out[(size_t)b * S + k] = ref;
        }
    }
    free(list);
    free(first);
    return exact ? OR_OK : OR_NONEXACT;
}

/*
 * Dense weight matrix W [N][N] (row = pre, column = post, §2.1), every synapse
 * of delay 1: the literal matrix form "spike vector of the previous step times
 * the weight matrix".  Same state layout as or_lif_sparse.
 */
int or_lif_dense(int32_t N, int32_t B, int32_t T,
                 const double* theta, const double* leak, const double* reset,
                 const int32_t* refractory, const double* amplitude,
                 const double* W, const uint8_t* ext, uint8_t* spikes,
                 double* V_out, int32_t* ref_out, int check_exact) {
    if (N < 1 || B < 1 || T < 0) return OR_EINVAL;
    int exact = 1;
    if (check_exact) {
        if (!check_params(N, theta, leak, reset, refractory, amplitude)) exact = 0;
    }
    double* in_abs = (double*)calloc((size_t)N, sizeof(double));
    double* U = (double*)malloc((size_t)N * sizeof(double));
    if (!in_abs || !U) { free(in_abs); free(U); return OR_ENOMEM; }
    for (int32_t i = 0; i < N; ++i)
        for (int32_t j = 0; j < N; ++j) {
            double x = W[(size_t)i * N + j];
            if (!isfinite(x)) { free(in_abs); free(U); return OR_EINVAL; }
            if (check_exact && x != 0.0 && !on_grid(x)) exact = 0;
            in_abs[j] += fabs(x);
        }

    for (int32_t b = 0; b < B; ++b) {
        double* V = V_out + (size_t)b * N;
        int32_t* ref = ref_out + (size_t)b * N;
        const uint8_t* xb = ext + (size_t)b * T * N;
        uint8_t* sb = spikes + (size_t)b * T * N;
        for (int32_t j = 0; j < N; ++j) { V[j] = reset[j]; ref[j] = 0; }

        for (int32_t t = 0; t < T; ++t) {
            for (int32_t j = 0; j < N; ++j) {
                U[j] = apply_leak(V[j], reset[j], leak[j]);
                if (check_exact && !(fabs(U[j]) + in_abs[j] + fabs(amplitude[j]) < EXACT_LIMIT))
                    exact = 0;
            }
            /* s(t-1) x W: a zero spike contributes exactly nothing */
            if (t > 0) {
                const uint8_t* sp = sb + (size_t)(t - 1) * N;
                for (int32_t i = 0; i < N; ++i) {
                    if (!sp[i]) continue;
                    const double* row = W + (size_t)i * N;
                    for (int32_t j = 0; j < N; ++j) U[j] += row[j];
                }
            }
            for (int32_t j = 0; j < N; ++j)
                if (xb[(size_t)t * N + j]) U[j] += amplitude[j];
            for (int32_t j = 0; j < N; ++j)
                sb[(size_t)t * N + j] =
                    (uint8_t)fire_and_reset(U[j], theta[j], reset[j], refractory[j], &V[j], &ref[j]);
        }
    }
    free(in_abs);
    free(U);
    return exact ? OR_OK : OR_NONEXACT;
}

/*
 * Surrogate-gradient backpropagation through time for a recurrent LIF layer
 * (the model above with delay-1 recurrent weights W_rec [N][N], external
 * input through W_in [Nin][N], no refractory period):
 *   U_t = leak(V_{t-1}) + s_{t-1} W_rec + x_t W_in
 *   s_t = H(U_t - theta)           (relaxed: s~(U_t - theta), see below)
 *   V_t = (1 - s_t) U_t + s_t r
 * Loss: L = mean over (b, j) of (c_bj / T - target_j)^2 with c_bj = sum_t s_t.
 * Threshold derivative (the "fast sigmoid" surrogate of slope k):
 *   ds/dU := 1 / (1 + k |U - theta|)^2,
 * which is the exact derivative of s~(x) = 1/2 + x / (1 + k|x|), a sigmoid
 * step of range (1/2 - 1/k, 1/2 + 1/k).  relaxed != 0 runs the forward with
 * s~ instead of H, so the returned gradient is then the true gradient of
 * that forward.
 * The leak is differentiated as 1 where it is not clamped (|V - r| > lambda),
 * 0 where it is.  Gradients are accumulated into dW_rec, dW_in (zeroed here).
 */
static double surrogate(double x, double k) {
    double d = 1.0 + k * fabs(x);
    return 1.0 / (d * d);
}

static double relaxed_spike(double x, double k) {
    return 0.5 + x / (1.0 + k * fabs(x));
}

int or_bptt(int32_t N, int32_t Nin, int32_t B, int32_t T, double theta, double lambda, double r,
            double k, int relaxed, const double* W_rec, const double* W_in, const uint8_t* x,
            const double* target, double* loss, double* dW_rec, double* dW_in, double* counts) {
    if (N < 1 || Nin < 0 || B < 1 || T < 1) return OR_EINVAL;
    size_t S = (size_t)T * B * N;
    double* U = (double*)malloc(S * sizeof(double));
    double* s = (double*)malloc(S * sizeof(double));
    double* V = (double*)malloc(S * sizeof(double));
    double* gU = (double*)calloc((size_t)B * N, sizeof(double));
    double* gUn = (double*)malloc((size_t)B * N * sizeof(double));
    if (!U || !s || !V || !gU || !gUn) {
        free(U); free(s); free(V); free(gU); free(gUn);
        return OR_ENOMEM;
    }
    /* forward */
    for (int32_t t = 0; t < T; ++t) {
        for (int32_t b = 0; b < B; ++b) {
            double* Ut = U + ((size_t)t * B + b) * N;
            for (int32_t j = 0; j < N; ++j)
                Ut[j] = apply_leak(t > 0 ? V[((size_t)(t - 1) * B + b) * N + j] : r, r, lambda);
            if (t > 0) {
                const double* sp = s + ((size_t)(t - 1) * B + b) * N;
                for (int32_t i = 0; i < N; ++i) {
                    if (sp[i] == 0.0) continue;
                    for (int32_t j = 0; j < N; ++j) Ut[j] += sp[i] * W_rec[(size_t)i * N + j];
                }
            }
            const uint8_t* xt = x + ((size_t)t * B + b) * Nin;
            for (int32_t i = 0; i < Nin; ++i) {
                if (!xt[i]) continue;
                for (int32_t j = 0; j < N; ++j) Ut[j] += W_in[(size_t)i * N + j];
            }
            double* st = s + ((size_t)t * B + b) * N;
            double* Vt = V + ((size_t)t * B + b) * N;
            for (int32_t j = 0; j < N; ++j) {
                st[j] = relaxed ? relaxed_spike(Ut[j] - theta, k) : (Ut[j] > theta ? 1.0 : 0.0);
                Vt[j] = (1.0 - st[j]) * Ut[j] + st[j] * r;
            }
        }
    }
    /* loss and its derivative with respect to every s_t (the same for all t) */
    double L = 0.0;
    for (int32_t b = 0; b < B; ++b)
        for (int32_t j = 0; j < N; ++j) {
            double c = 0.0;
            for (int32_t t = 0; t < T; ++t) c += s[((size_t)t * B + b) * N + j];
            counts[(size_t)b * N + j] = c;
            double e = c / T - target[j];
            L += e * e;
        }
    *loss = L / ((double)B * N);
    for (size_t q = 0; q < (size_t)N * N; ++q) dW_rec[q] = 0.0;
    for (size_t q = 0; q < (size_t)Nin * N; ++q) dW_in[q] = 0.0;
    /* backward: gU holds dL/dU_{t+1} (zero beyond the last step) */
    for (int32_t t = T - 1; t >= 0; --t) {
        for (int32_t b = 0; b < B; ++b) {
            const double* Ut = U + ((size_t)t * B + b) * N;
            const double* st = s + ((size_t)t * B + b) * N;
            const double* Vt = V + ((size_t)t * B + b) * N;
            const double* gnext = gU + (size_t)b * N;
            double* gcur = gUn + (size_t)b * N;
            for (int32_t i = 0; i < N; ++i) {
                /* dL/ds_t: through the loss and through s_t W_rec into U_{t+1} */
                double a = 2.0 * (counts[(size_t)b * N + i] / T - target[i]) / ((double)B * N * T);
                for (int32_t j = 0; j < N; ++j) a += gnext[j] * W_rec[(size_t)i * N + j];
                /* dL/dV_t: through leak(V_t) into U_{t+1} */
                double gv = fabs(Vt[i] - r) > lambda ? gnext[i] : 0.0;
                double sg = surrogate(Ut[i] - theta, k);
                gcur[i] = a * sg + gv * ((1.0 - st[i]) + (r - Ut[i]) * sg);
            }
        }
        /* weight gradients: U_t = ... + s_{t-1} W_rec + x_t W_in */
        for (int32_t b = 0; b < B; ++b) {
            const double* gcur = gUn + (size_t)b * N;
            if (t > 0) {
                const double* sp = s + ((size_t)(t - 1) * B + b) * N;
                for (int32_t i = 0; i < N; ++i) {
                    if (sp[i] == 0.0) continue;
                    for (int32_t j = 0; j < N; ++j) dW_rec[(size_t)i * N + j] += sp[i] * gcur[j];
                }
            }
            const uint8_t* xt = x + ((size_t)t * B + b) * Nin;
            for (int32_t i = 0; i < Nin; ++i) {
                if (!xt[i]) continue;
                for (int32_t j = 0; j < N; ++j) dW_in[(size_t)i * N + j] += gcur[j];
            }
        }
        double* tmp = gU; gU = gUn; gUn = tmp;
    }
    free(U); free(s); free(V); free(gU); free(gUn);
    return OR_OK;
}
