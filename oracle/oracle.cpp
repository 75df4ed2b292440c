// FP64 CPU oracle for the 360Roam geometry-aware radiance-field hot path.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or calls
// this file; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark do. It is plain and slow on purpose: loops in the order of the
// paper's definitions, no blocking, no fusion, no reordering. It shares no
// code with the HIP library.
//
// Paper: "360Roam: Real-Time Indoor Roaming Using Geometry-Aware 360°
// Radiance Fields" (arXiv 2208.02705). Equation numbers below count the
// paper's displayed equations in order: Eq.1 the two-stage MLP (Sec. 3.1),
// Eq.2 pixel <-> sphere and Eq.3 sphere -> Cartesian (Sec. 3.2), Eq.4 colour
// and depth compositing and Eq.5 the sample weights (Sec. 3.2), Eq.6 the
// logit occupancy update (Sec. 4.1), Eq.7 the distillation loss (Sec. 4.2).
//
// Precision: the geometric front end (ray directions, voxel traversal,
// sample positions) is a specified FP32 formula, evaluated here in float
// with correctly rounded operations and no contraction (build with
// -ffp-contract=off, no fast-math), so that sample -> voxel -> field
// assignment can be compared bit for bit. Everything after the sample
// position (encoding, MLP, compositing, loss, gradients) is FP64.
//
// Parity pins: every function below is checked by the CPU test-suite against
// closed forms, invariants or brute force (see tests/test_oracle_pins.py).
// The absolute values of rendered pixels are not printed in the paper, so
// end-to-end pixel values are pinned only through those per-stage checks.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>
#include <limits>

// Test-only switch: the mutation tests rebuild this file with ORC_PLANT = k
// to plant a known mistake and check that the pins catch it. 0 = none.
#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

namespace {

// ---------------------------------------------------------------------------
// Scene description (mirrors the ctypes structure in oracle/__init__.py)
// ---------------------------------------------------------------------------
struct OrcScene {
    int32_t n[3];          // voxels per axis
    float lo[3];           // grid lower corner (m)
    float voxel;           // voxel edge (m); a power of two
    float threshold;       // occupied where occ > threshold
    const float* occ;      // [n2][n1][n0], x fastest
    const int32_t* field;  // same layout, -1 = none
    int32_t n_fields;
    int32_t hidden;
    int32_t L_xyz, L_dir;
    float center[3];       // encoding centre
    float half_extent;     // encoding half extent: xhat = (p - center) / half_extent
    const float* weights;  // [n_fields][P] canonical FP32
    float near_, far_;
    int32_t max_samples;
    int32_t samples_per_voxel; // k >= 1 samples per occupied segment (0 reads as 1)
    const float* frames;       // optional [n_fields][4]: per-field encoding centre (3) and half extent
};

const double PI = 3.14159265358979323846;

// sin(pi r) in FP64 with the argument reduced exactly: r mod 2 is exact in
// binary floating point, and the symmetric fold keeps |r| <= 1/2 so that
// integer r gives exactly 0 and half-integers give exactly +-1.
double sinpi_d(double r) {
    double m = std::fmod(r, 2.0);        // exact, in (-2, 2)
    if (m > 1.0) m -= 2.0;               // exact, now in [-1, 1]
    if (m < -1.0) m += 2.0;
    if (m > 0.5) m = 1.0 - m;            // sin(pi m) = sin(pi (1 - m))
    else if (m < -0.5) m = -1.0 - m;     // sin(pi m) = sin(pi (-1 - m))
    return std::sin(PI * m);
}
double cospi_d(double r) { return sinpi_d(r + 0.5); }  // r + 1/2 is exact here

// ---------------------------------------------------------------------------
// Ray generation (Sec. 3.2, Eq.2 and Eq.3)
// ---------------------------------------------------------------------------
// Eq.2 maps longitude phi and latitude theta to pixel (u, v); inverted at
// the pixel centre (u + 1/2, v + 1/2):
//   phi   = pi * a_phi,   a_phi   = ((2u + 1) - W) / W
//   theta = pi * a_theta, a_theta = (H - (2v + 1)) / (2H)
// each a correctly rounded FP32 division of exact integers. The sines and
// cosines are evaluated in FP64 and rounded once to FP32.
// Eq.3: d = (cos(theta) sin(phi), -sin(theta), cos(theta) cos(phi)),
// camera frame x right, y down, z forward; FP32 products, not renormalised.
void equirect_trig(int W, int H, int u, int v, float* sphi, float* cphi, float* sth, float* cth) {
    float a_phi = (float)((2 * u + 1) - W) / (float)W;
    float a_th = (float)(H - (2 * v + 1)) / (float)(2 * H);
    *sphi = (float)sinpi_d((double)a_phi);
    *cphi = (float)cospi_d((double)a_phi);
    *sth = (float)sinpi_d((double)a_th);
    *cth = (float)cospi_d((double)a_th);
}

// World direction d = R d_cam with the chain fma(R2, z, fma(R1, y, R0 * x)).
void to_world(const float* c2w, const float dc[3], float o[3], float d[3]) {
    for (int i = 0; i < 3; ++i) {
        const float* r = c2w + 4 * i;
        d[i] = std::fma(r[2], dc[2], std::fma(r[1], dc[1], r[0] * dc[0]));
        o[i] = r[3];
    }
}

// ---------------------------------------------------------------------------
// Occupancy-grid sampling: voxel traversal in FP32 (Sec. 4.2: fine-tuning
// samples densely inside the occupied voxels; Sec. 5: rays are cast over the
// labelled occupancy map). One midpoint sample per occupied voxel segment, with the
// segment length as its interval, the first max_samples in increasing t.
// ---------------------------------------------------------------------------
struct Seg { float t_mid, delta; int32_t voxel, field; };

// The FP32 voxel walk shared by the sampler and the occupancy update: visits
// the voxels the ray crosses between t0 = max(near, box entry) and t1 =
// min(far, box exit) in increasing t and calls fn(lin, t_in, t_out) for every
// segment of positive length (zero-length edge and corner touches are
// skipped); fn returns false to stop the walk.
template <class F>
void walk_ray(const int32_t n[3], const float lo[3], float voxel, float near_, float far_, const float o[3],
              const float d[3], F fn) {
    const float INF = std::numeric_limits<float>::infinity();
    float inv[3], hi[3];
    bool active[3];
    float t0 = near_, t1 = far_;
    for (int a = 0; a < 3; ++a) {
        hi[a] = lo[a] + (float)n[a] * voxel;
        active[a] = d[a] != 0.0f;
        if (active[a]) {
            inv[a] = 1.0f / d[a];
            float ta = (lo[a] - o[a]) * inv[a];
            float tb = (hi[a] - o[a]) * inv[a];
            t0 = std::max(t0, std::min(ta, tb));
            t1 = std::min(t1, std::max(ta, tb));
        } else {
            inv[a] = 0.0f;
            if (!(o[a] >= lo[a] && o[a] < hi[a])) return;
        }
    }
    if (!(t0 < t1)) return;
    const float inv_vox = 1.0f / voxel;   // exact: the voxel edge is a power of two
    int idx[3];
    for (int a = 0; a < 3; ++a) {
        float p = std::fma(t0, d[a], o[a]);
        float q = (p - lo[a]) * inv_vox;
        float fq = std::floor(q);
        int i = (int)fq;
        if (q == fq && d[a] < 0.0f) i -= 1;   // on a plane moving down: the lower voxel
        idx[a] = std::min(std::max(i, 0), n[a] - 1);
    }
    float t_in = t0;
    for (;;) {
        float tn[3];
        for (int a = 0; a < 3; ++a) {
            if (active[a]) {
                float plane = std::fma((float)(idx[a] + (d[a] > 0.0f ? 1 : 0)), voxel, lo[a]);
                tn[a] = (plane - o[a]) * inv[a];
            } else {
                tn[a] = INF;
            }
        }
        int am = 0;                           // ties go to the lowest axis
        if (tn[1] < tn[am]) am = 1;
        if (tn[2] < tn[am]) am = 2;
        float t_out = std::min(tn[am], t1);
        int64_t lin = idx[0] + (int64_t)n[0] * (idx[1] + (int64_t)n[1] * idx[2]);
        if (t_out > t_in && !fn(lin, t_in, t_out)) break;
        if (!(tn[am] < t1)) break;
        t_in = std::max(t_in, tn[am]);
        idx[am] += d[am] > 0.0f ? 1 : -1;
        if (idx[am] < 0 || idx[am] >= n[am]) break;
    }
}

// With k samples per occupied segment, the segment is cut at b_j = fma(j,
// (t_out - t_in) / k, t_in) for 0 < j < k (b_0 = t_in, b_k = t_out) and each
// piece gives its midpoint (b_j + b_j+1) / 2 with interval b_j+1 - b_j; k = 1
// is the single midpoint sample.
int sample_ray(const OrcScene& s, const float o[3], const float d[3], Seg* out) {
    const float far_ = ORC_PLANT == 9 ? std::numeric_limits<float>::infinity() : s.far_;
    const int k = s.samples_per_voxel > 1 ? s.samples_per_voxel : 1;
    int count = 0;
    walk_ray(s.n, s.lo, s.voxel, s.near_, far_, o, d, [&](int64_t lin, float t_in, float t_out) {
        if (s.occ[lin] > s.threshold && s.field[lin] >= 0) {
            const float piece = (t_out - t_in) / (float)k;
            float b0 = t_in;
            for (int j = 0; j < k; ++j) {
                const float b1 = j + 1 == k ? t_out : std::fma((float)(j + 1), piece, t_in);
                out[count].t_mid = ORC_PLANT == 8 ? b1 : (ORC_PLANT == 23 && k > 1 ? b0 : (b0 + b1) * 0.5f);
                out[count].delta = b1 - b0;
                out[count].voxel = (int32_t)lin;
                out[count].field = s.field[lin];
                b0 = b1;
                if (++count == s.max_samples) return false;
            }
        }
        return true;
    });
    return count;
}

// Encoding input: p = fma(t_mid, d, o), xhat = (p - center) * (1 / half_extent)
// in FP32, then widened exactly.
// With per-field frames, field f uses its own centre c_f and half extent h_f:
// xhat = (p - c_f) * (1 / h_f).
void sample_position(const OrcScene& s, const float o[3], const float d[3], float t_mid, int field, double xh[3]) {
    const bool own = s.frames && ORC_PLANT != 25;
    const float* c = own ? s.frames + 4 * field : s.center;
    const float inv_h = 1.0f / (own ? s.frames[4 * field + 3] : s.half_extent);
    for (int a = 0; a < 3; ++a) {
        float p = std::fma(t_mid, d[a], o[a]);
        xh[a] = (double)((p - c[a]) * inv_h);
    }
}

// ---------------------------------------------------------------------------
// Positional encoding (Sec. 3.1, applied to each component separately):
//   gamma_L(x) = [x, sin(2^0 pi x), cos(2^0 pi x), ..., sin(2^(L-1) pi x), cos(...)]
// laid out as the three raw components, then for each frequency l the sines
// of (x, y, z) followed by the cosines of (x, y, z). Width 3 + 6L.
// ---------------------------------------------------------------------------
void encode(const double x[3], int L, double* out) {
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2];
    for (int l = 0; l < L; ++l) {
        for (int c = 0; c < 3; ++c) {
            double r = std::ldexp(x[c], ORC_PLANT == 4 ? l + 1 : l);   // 2^l x, exact
            out[3 + 6 * l + c] = ORC_PLANT == 3 ? cospi_d(r) : sinpi_d(r);
            out[3 + 6 * l + 3 + c] = cospi_d(r);
        }
    }
}

double softplus(double z) { return std::max(z, 0.0) + std::log1p(std::exp(-std::fabs(z))); }
double sigmoid(double z) { return 1.0 / (1.0 + std::exp(-z)); }
double relu(double z) { return z > 0.0 ? z : 0.0; }

// y[o] = b[o] + sum_i W[o][i] x[i]   (W row-major [out x in])
void dense(const double* W, const double* b, int n_out, int n_in, const double* x, double* y) {
    for (int o = 0; o < n_out; ++o) {
        double acc = b[o];
        for (int i = 0; i < n_in; ++i)
            acc += (ORC_PLANT == 5 && n_out == n_in ? W[(size_t)i * n_in + o] : W[(size_t)o * n_in + i]) * x[i];
        y[o] = acc;
    }
}

// Views of one local field's canonical parameter vector.
struct LocalNet {
    const double *W1, *b1, *W2, *b2, *ws, *bs, *Wf, *bf, *W3, *b3, *W4, *b4;
    int h, dx, dd;
};
size_t local_params(int h, int dx, int dd) {
    return (size_t)h * dx + h + (size_t)h * h + h + h + 1 + (size_t)h * h + h + (size_t)h * (h + dd) + h + 3 * (size_t)h + 3;
}
LocalNet local_view(const double* w, int h, int dx, int dd) {
    LocalNet n; n.h = h; n.dx = dx; n.dd = dd;
    const double* p = w;
    n.W1 = p; p += (size_t)h * dx; n.b1 = p; p += h;
    n.W2 = p; p += (size_t)h * h;  n.b2 = p; p += h;
    n.ws = p; p += h;              n.bs = p; p += 1;
    n.Wf = p; p += (size_t)h * h;  n.bf = p; p += h;
    n.W3 = p; p += (size_t)h * (h + dd); n.b3 = p; p += h;
    n.W4 = p; p += 3 * (size_t)h;  n.b4 = p;
    return n;
}

// Activations of one local-field evaluation, kept for the backward pass.
struct LocalAct {
    std::vector<double> gx, gd, z1, h1, z2, h2, f, in3, z3, h3;
    double zs, sigma, z4[3], rgb[3];
};

// Local field MLP (Eq.1, tiny form): h1 = relu(W1 gx + b1); h2 = relu(W2 h1 + b2);
// sigma = softplus(ws h2 + bs); f = Wf h2 + bf (linear);
// h3 = relu(W3 [f; gd] + b3); rgb = sigmoid(W4 h3 + b4).
void local_forward(const LocalNet& n, const double xh[3], const double dir[3], int Lx, int Ld, LocalAct& a) {
    const int h = n.h;
    a.gx.assign(n.dx, 0.0); a.gd.assign(n.dd, 0.0);
    encode(xh, Lx, a.gx.data());
    encode(dir, Ld, a.gd.data());
    a.z1.assign(h, 0.0); a.h1.assign(h, 0.0); a.z2.assign(h, 0.0); a.h2.assign(h, 0.0);
    a.f.assign(h, 0.0); a.in3.assign(h + n.dd, 0.0); a.z3.assign(h, 0.0); a.h3.assign(h, 0.0);
    dense(n.W1, n.b1, h, n.dx, a.gx.data(), a.z1.data());
    for (int i = 0; i < h; ++i) a.h1[i] = relu(a.z1[i]);
    dense(n.W2, n.b2, h, h, a.h1.data(), a.z2.data());
    for (int i = 0; i < h; ++i) a.h2[i] = ORC_PLANT == 6 ? a.z2[i] : relu(a.z2[i]);
    dense(n.ws, n.bs, 1, h, a.h2.data(), &a.zs);
    a.sigma = ORC_PLANT == 7 ? relu(a.zs) : softplus(a.zs);
    dense(n.Wf, n.bf, h, h, a.h2.data(), a.f.data());
    if (ORC_PLANT == 26) for (int i = 0; i < h; ++i) a.f[i] = relu(a.f[i]);
    for (int i = 0; i < h; ++i) a.in3[i] = a.f[i];
    for (int i = 0; i < n.dd; ++i) a.in3[h + i] = a.gd[i];
    dense(n.W3, n.b3, h, h + n.dd, a.in3.data(), a.z3.data());
    for (int i = 0; i < h; ++i) a.h3[i] = relu(a.z3[i]);
    dense(n.W4, n.b4, 3, h, a.h3.data(), a.z4);
    for (int c = 0; c < 3; ++c) a.rgb[c] = sigmoid(a.z4[c]);
}

// dW += g x^T, db += g; dx = W^T g (dx may be null)
void dense_backward(const double* W, int n_out, int n_in, const double* x, const double* g,
                    double* dW, double* db, double* dx) {
    for (int o = 0; o < n_out; ++o) {
        for (int i = 0; i < n_in; ++i) dW[(size_t)o * n_in + i] += g[o] * x[i];
        db[o] += g[o];
    }
    if (dx) {
        for (int i = 0; i < n_in; ++i) {
            double acc = 0.0;
            for (int o = 0; o < n_out; ++o) acc += W[(size_t)o * n_in + i] * g[o];
            dx[i] = acc;
        }
    }
}

// Backward of local_forward given dL/dsigma and dL/drgb; accumulates into the
// gradient view `gn` (same layout as the weights).
void local_backward(const LocalNet& n, const LocalAct& a, double dsigma, const double drgb[3], const LocalNet& gn) {
    const int h = n.h;
    double dz4[3];
    for (int c = 0; c < 3; ++c) dz4[c] = drgb[c] * a.rgb[c] * (1.0 - a.rgb[c]);
    std::vector<double> dh3(h), dz3(h), din3(h + n.dd), dh2(h, 0.0), dz2(h), dh1(h), dz1(h), tmp(h);
    dense_backward(n.W4, 3, h, a.h3.data(), dz4, (double*)gn.W4, (double*)gn.b4, dh3.data());
    for (int i = 0; i < h; ++i) dz3[i] = a.z3[i] > 0.0 ? dh3[i] : 0.0;
    dense_backward(n.W3, h, h + n.dd, a.in3.data(), dz3.data(), (double*)gn.W3, (double*)gn.b3, din3.data());
    // f = Wf h2 + bf (linear): df = din3[0:h]
    if (ORC_PLANT == 26) for (int i = 0; i < h; ++i) if (!(a.f[i] > 0.0)) din3[i] = 0.0;
    dense_backward(n.Wf, h, h, a.h2.data(), din3.data(), (double*)gn.Wf, (double*)gn.bf, tmp.data());
    for (int i = 0; i < h; ++i) dh2[i] += tmp[i];
    double dzs = dsigma * sigmoid(a.zs);   // softplus' = sigmoid
    dense_backward(n.ws, 1, h, a.h2.data(), &dzs, (double*)gn.ws, (double*)gn.bs, tmp.data());
    for (int i = 0; i < h; ++i) dh2[i] += tmp[i];
    for (int i = 0; i < h; ++i) dz2[i] = a.z2[i] > 0.0 ? dh2[i] : 0.0;
    dense_backward(n.W2, h, h, a.h1.data(), dz2.data(), (double*)gn.W2, (double*)gn.b2, dh1.data());
    for (int i = 0; i < h; ++i) dz1[i] = a.z1[i] > 0.0 ? dh1[i] : 0.0;
    dense_backward(n.W1, h, n.dx, a.gx.data(), dz1.data(), (double*)gn.W1, (double*)gn.b1, nullptr);
}

// Magnitudes for error bounds (running error analysis): each quantity of the
// local-field forward and backward re-evaluated with the absolute value of
// every operand, so that |q| <= q_mag by the triangle inequality and a
// rounding of relative size u in any term moves q by at most u q_mag. ReLU
// masks and the slopes of softplus and sigmoid are those of the actual
// evaluation `a`. dsig_mag >= 0 and drgb_mag[3] >= 0 are the magnitudes of
// dL/dsigma and dL/drgb; magnitudes of the weight gradients accumulate into gm.
// Kinks: a ReLU unit whose pre-activation lies within tau of zero may take
// the other branch in a computation whose pre-activations carry errors up to
// tau; the flip adds or drops the unit's whole term (its row and bias, and
// the path below it) for that sample. gk (optional) accumulates, for every
// such unit, the magnitude of that term: the backward of the magnitudes
// seeded with the unit's incoming gradient magnitude alone.
void dense_abs(const double* W, const double* b, int n_out, int n_in, const double* x, double* y) {
    for (int o = 0; o < n_out; ++o) {
        double acc = std::fabs(b[o]);
        for (int i = 0; i < n_in; ++i) acc += std::fabs(W[(size_t)o * n_in + i]) * x[i];
        y[o] = acc;
    }
}
void dense_backward_abs(const double* W, int n_out, int n_in, const double* x, const double* g,
                        double* dW, double* db, double* dx) {
    for (int o = 0; o < n_out; ++o) {
        for (int i = 0; i < n_in; ++i) dW[(size_t)o * n_in + i] += g[o] * x[i];
        db[o] += g[o];
    }
    if (dx) {
        for (int i = 0; i < n_in; ++i) {
            double acc = 0.0;
            for (int o = 0; o < n_out; ++o) acc += std::fabs(W[(size_t)o * n_in + i]) * g[o];
            dx[i] = acc;
        }
    }
}
void local_magnitude(const LocalNet& n, const LocalAct& a, double dsig_mag, const double drgb_mag[3],
                     const LocalNet& gm, double tau, const LocalNet* gk) {
    const int h = n.h;
    std::vector<double> gx(n.dx), z1(h), h1(h), z2(h), h2(h), f(h), in3(h + n.dd), z3(h), h3(h);
    std::vector<char> m1(h), m2(h), m3(h);
    for (int i = 0; i < n.dx; ++i) gx[i] = std::fabs(a.gx[i]);
    dense_abs(n.W1, n.b1, h, n.dx, gx.data(), z1.data());
    for (int i = 0; i < h; ++i) { m1[i] = a.z1[i] > 0.0; h1[i] = m1[i] ? z1[i] : 0.0; }
    dense_abs(n.W2, n.b2, h, h, h1.data(), z2.data());
    for (int i = 0; i < h; ++i) { m2[i] = a.z2[i] > 0.0; h2[i] = m2[i] ? z2[i] : 0.0; }
    dense_abs(n.Wf, n.bf, h, h, h2.data(), f.data());
    for (int i = 0; i < h; ++i) in3[i] = f[i];
    for (int i = 0; i < n.dd; ++i) in3[h + i] = std::fabs(a.gd[i]);
    dense_abs(n.W3, n.b3, h, h + n.dd, in3.data(), z3.data());
    for (int i = 0; i < h; ++i) { m3[i] = a.z3[i] > 0.0; h3[i] = m3[i] ? z3[i] : 0.0; }

    double dz4[3];
    for (int c = 0; c < 3; ++c) dz4[c] = drgb_mag[c] * a.rgb[c] * (1.0 - a.rgb[c]);
    std::vector<double> dh3(h), dz3(h), din3(h + n.dd), dh2(h, 0.0), dz2(h), dh1(h), dz1(h), tmp(h);
    dense_backward_abs(n.W4, 3, h, h3.data(), dz4, (double*)gm.W4, (double*)gm.b4, dh3.data());
    for (int i = 0; i < h; ++i) dz3[i] = m3[i] ? dh3[i] : 0.0;
    dense_backward_abs(n.W3, h, h + n.dd, in3.data(), dz3.data(), (double*)gm.W3, (double*)gm.b3, din3.data());
    dense_backward_abs(n.Wf, h, h, h2.data(), din3.data(), (double*)gm.Wf, (double*)gm.bf, tmp.data());
    for (int i = 0; i < h; ++i) dh2[i] += tmp[i];
    double dzs = dsig_mag * sigmoid(a.zs);
    dense_backward_abs(n.ws, 1, h, h2.data(), &dzs, (double*)gm.ws, (double*)gm.bs, tmp.data());
    for (int i = 0; i < h; ++i) dh2[i] += tmp[i];
    for (int i = 0; i < h; ++i) dz2[i] = m2[i] ? dh2[i] : 0.0;
    dense_backward_abs(n.W2, h, h, h1.data(), dz2.data(), (double*)gm.W2, (double*)gm.b2, dh1.data());
    for (int i = 0; i < h; ++i) dz1[i] = m1[i] ? dh1[i] : 0.0;
    dense_backward_abs(n.W1, h, n.dx, gx.data(), dz1.data(), (double*)gm.W1, (double*)gm.b1, nullptr);
    if (!gk) return;

    // terms through units within tau of their kink: seeds at layer 3, then the
    // path below it joined by the seeds of layers 2 and 1 (all linear in the seeds)
    std::vector<double> k3(h, 0.0), kin3(h + n.dd), kh2(h), kz2(h), kh1(h), kz1(h);
    bool any = false;
    for (int i = 0; i < h; ++i)
        if (std::fabs(a.z3[i]) <= tau) { k3[i] = dh3[i]; any = true; }
    dense_backward_abs(n.W3, h, h + n.dd, in3.data(), k3.data(), (double*)gk->W3, (double*)gk->b3, kin3.data());
    dense_backward_abs(n.Wf, h, h, h2.data(), kin3.data(), (double*)gk->Wf, (double*)gk->bf, kh2.data());
    for (int i = 0; i < h; ++i) {
        kz2[i] = m2[i] ? kh2[i] : 0.0;
        if (std::fabs(a.z2[i]) <= tau) { kz2[i] += dh2[i]; any = true; }
    }
    dense_backward_abs(n.W2, h, h, h1.data(), kz2.data(), (double*)gk->W2, (double*)gk->b2, kh1.data());
    for (int i = 0; i < h; ++i) {
        kz1[i] = m1[i] ? kh1[i] : 0.0;
        if (std::fabs(a.z1[i]) <= tau) { kz1[i] += dh1[i]; any = true; }
    }
    dense_backward_abs(n.W1, h, n.dx, gx.data(), kz1.data(), (double*)gk->W1, (double*)gk->b1, nullptr);
    (void)any;
}

// ---------------------------------------------------------------------------
// Compositing (Sec. 3.2, Eq.4 and Eq.5): with tau_k = sigma_k delta_k,
//   w_i = exp(-sum_{k<i} tau_k) (1 - exp(-tau_i)),
//   C = sum_i w_i c_i, D = sum_i w_i t_i, A = sum_i w_i.
// No background colour is added.
// ---------------------------------------------------------------------------
void composite(int n, const double* sigma, const double* rgb /*[n][3]*/, const double* t_mid,
               const double* delta, double C[3], double* D, double* A, double* w_out) {
    C[0] = C[1] = C[2] = 0.0; *D = 0.0; *A = 0.0;
    double S = 0.0;   // sum_{k<i} tau_k
    for (int i = 0; i < n; ++i) {
        double tau = sigma[i] * delta[i];
        double w = (ORC_PLANT == 1 ? 1.0 : std::exp(ORC_PLANT == 2 ? -(S + tau) : -S)) * (-std::expm1(-tau));
        if (w_out) w_out[i] = w;
        for (int c = 0; c < 3; ++c) C[c] += w * rgb[3 * i + c];
        *D += w * t_mid[i];
        *A += w;
        S += tau;
    }
}

// Gradient of C w.r.t. sigma_i and c_i, from dL/dC = g:
//   dL/dc_i = w_i g,
//   dL/dsigma_i = delta_i [ T_{i+1} (c_i . g) - ((C - C_{<=i}) . g) ],
// where T_{i+1} = exp(-sum_{k<=i} tau_k) and C_{<=i} = sum_{k<=i} w_k c_k.
void composite_backward(int n, const double* sigma, const double* rgb, const double* delta,
                        const double g[3], double* dsigma, double* drgb) {
    std::vector<double> w(n);
    double C[3] = {0, 0, 0};
    double S = 0.0;
    for (int i = 0; i < n; ++i) {
        double tau = sigma[i] * delta[i];
        w[i] = std::exp(-S) * (-std::expm1(-tau));
        for (int c = 0; c < 3; ++c) C[c] += w[i] * rgb[3 * i + c];
        S += tau;
    }
    double Cle[3] = {0, 0, 0};
    S = 0.0;
    for (int i = 0; i < n; ++i) {
        double tau = sigma[i] * delta[i];
        S += tau;
        double T_next = std::exp(-S);
        double cg = 0.0, rg = 0.0;
        for (int c = 0; c < 3; ++c) {
            Cle[c] += w[i] * rgb[3 * i + c];
            cg += rgb[3 * i + c] * g[c];
            rg += (C[c] - Cle[c]) * g[c];
            drgb[3 * i + c] = w[i] * g[c];
        }
        dsigma[i] = delta[i] * (T_next * cg + (ORC_PLANT == 10 ? rg : -rg));
    }
}

// Magnitudes of the compositing gradients (see local_magnitude): with
// colours, weights and transmittances non-negative and gm[c] >= |dL/dC_c|,
//   drgb_mag_i = w_i gm,
//   dsig_mag_i = delta_i [T_{i+1} (c_i . gm) + ((C + C_{<=i}) . gm)],
// the tail C - C_{<=i} taken at the magnitude of its two sums.
void composite_magnitude(int n, const double* sigma, const double* rgb, const double* delta, const double gm[3],
                         double* dsig_mag, double* drgb_mag) {
    std::vector<double> w(n);
    double C[3] = {0, 0, 0};
    double S = 0.0;
    for (int i = 0; i < n; ++i) {
        double tau = sigma[i] * delta[i];
        w[i] = std::exp(-S) * (-std::expm1(-tau));
        for (int c = 0; c < 3; ++c) C[c] += w[i] * rgb[3 * i + c];
        S += tau;
    }
    double Cle[3] = {0, 0, 0};
    S = 0.0;
    for (int i = 0; i < n; ++i) {
        S += sigma[i] * delta[i];
        double cg = 0.0, rg = 0.0;
        for (int c = 0; c < 3; ++c) {
            Cle[c] += w[i] * rgb[3 * i + c];
            cg += rgb[3 * i + c] * gm[c];
            rg += (C[c] + Cle[c]) * gm[c];
            drgb_mag[3 * i + c] = w[i] * gm[c];
        }
        dsig_mag[i] = delta[i] * (std::exp(-S) * cg + rg);
    }
}

// ---------------------------------------------------------------------------
// Stage I of Alg.1 (Sec. 4.1): the measurement a ray of the global field
// gives. With the Eq.5 weights w_i of its samples: opacity A = sum w_i;
// normalised weights v_i = w_i / A; depth D = sum v_i t_i (the Eq.4 depth
// over normalised weights); uncertainty U = sqrt(sum v_i (t_i - D)^2), the
// spread of the normalised weights about D. A ray with A = 0 gives D = U = 0.
// ---------------------------------------------------------------------------
void depth_stats(int n, const double* sigma, const double* t, const double* delta, double* D, double* U, double* A) {
    std::vector<double> w(n), rgb(3 * (size_t)n, 0.0);
    double C[3], Dw;
    composite(n, sigma, rgb.data(), t, delta, C, &Dw, A, w.data());
    *D = 0.0; *U = 0.0;
    if (!(*A > 0.0)) return;
    const double inv = ORC_PLANT == 16 ? 1.0 : 1.0 / *A;
    for (int i = 0; i < n; ++i) *D += w[i] * inv * t[i];
    double var = 0.0;
    for (int i = 0; i < n; ++i) var += w[i] * inv * (t[i] - *D) * (t[i] - *D);
    *U = std::sqrt(var);
}

// Stage I update for one sampling position (one pose): the logit form of
// Eq.6, logit(p | z_1:t) = logit(p | z_1:t-1) + logit(p | z_t), with an
// inverse sensor model read in the OctoMap manner the paper adopts:
//  - a ray is a measurement when A >= min_opacity and D, U are finite, U >= 0;
//  - walking its voxels (the sampler's FP32 walk, every voxel), a segment
//    that ends at or before D - U is free space (logit l_miss < 0); the voxel
//    whose segment [t_in, t_out) holds D is the hit, and the walk stops
//    there; voxels inside the uncertainty band get nothing;
//  - the hit's measurement logit shrinks with the ray's uncertainty:
//    h = l_hit / (1 + U / voxel), all FP32 (the measurement probability
//    follows the global field's own estimate);
//  - per pose every voxel takes at most one measurement: the largest hit
//    logit of the rays that end in it, otherwise l_miss if a ray passed
//    through it freely;
//  - the sum is clamped to [l_min, l_max] (Sec. 4.1: -2 and 3.5, i.e.
//    probability 0.12 to 0.97); voxels without a measurement keep their value.
// prob (optional) receives 1 / (1 + exp(-l)) for every voxel.
struct OrcOcc {
    int32_t n[3];
    float lo[3];
    float voxel;
    float near_, far_;
    float l_hit, l_miss, l_min, l_max;
    float min_opacity;
};

template <class F>
void parallel_for(int64_t n, int nthreads, F fn) {
    if (nthreads <= 1 || n < 2) { fn(0, n, 0); return; }
    std::vector<std::thread> th;
    int64_t chunk = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back(fn, b, e, t);
    }
    for (auto& x : th) x.join();
}

std::vector<double> widen(const float* w, size_t n) {
    std::vector<double> out(n);
    for (size_t i = 0; i < n; ++i) out[i] = (double)w[i];
    return out;
}

// Global omnidirectional field (360NeRF architecture table, Sec. 3.2): eight
// position layers of width W with [h4 ; gx] at the fifth layer input, the
// eighth without activation; sigma = relu(ws h8 + bs); f = relu(Wf h8 + bf);
// h10 = relu(W10 [f ; gd] + b10); rgb = sigmoid(W11 h10 + b11).
struct GlobalNet {
    const double* W[8]; const double* b[8];
    const double *ws, *bs, *Wf, *bf, *W10, *b10, *W11, *b11;
    int w, c, dx, dd;
};
size_t global_params(int w, int c, int dx, int dd) {
    return (size_t)w * dx + w + 3 * ((size_t)w * w + w) + (size_t)w * (w + dx) + w + 3 * ((size_t)w * w + w)
           + w + 1 + (size_t)w * w + w + (size_t)c * (w + dd) + c + 3 * (size_t)c + 3;
}
GlobalNet global_view(const double* p, int w, int c, int dx, int dd) {
    GlobalNet n; n.w = w; n.c = c; n.dx = dx; n.dd = dd;
    for (int k = 0; k < 8; ++k) {
        int in = (k == 0) ? dx : (k == 4 ? w + dx : w);
        n.W[k] = p; p += (size_t)w * in; n.b[k] = p; p += w;
    }
    n.ws = p; p += w; n.bs = p; p += 1;
    n.Wf = p; p += (size_t)w * w; n.bf = p; p += w;
    n.W10 = p; p += (size_t)c * (w + dd); n.b10 = p; p += c;
    n.W11 = p; p += 3 * (size_t)c; n.b11 = p;
    return n;
}
struct GlobalAct {
    std::vector<double> gx, gd, in[8], z[8], h[8], zf, f, in10, z10, h10;
    double zs, sigma, z11[3], rgb[3];
};
void global_forward(const GlobalNet& n, const double xh[3], const double dir[3], int Lx, int Ld, GlobalAct& a) {
    a.gx.assign(n.dx, 0.0); a.gd.assign(n.dd, 0.0);
    encode(xh, Lx, a.gx.data());
    encode(dir, Ld, a.gd.data());
    for (int k = 0; k < 8; ++k) {
        if (k == 0) a.in[k] = a.gx;
        else if (k == 4) {
            a.in[k] = a.h[3];
            a.in[k].insert(a.in[k].end(), a.gx.begin(), a.gx.end());
            if (ORC_PLANT == 12) for (int i = n.w; i < n.w + n.dx; ++i) a.in[k][i] = 0.0;
        }
        else a.in[k] = a.h[k - 1];
        a.z[k].assign(n.w, 0.0);
        dense(n.W[k], n.b[k], n.w, (int)a.in[k].size(), a.in[k].data(), a.z[k].data());
        a.h[k].assign(n.w, 0.0);
        for (int i = 0; i < n.w; ++i) a.h[k][i] = (k == 7) ? a.z[k][i] : relu(a.z[k][i]);
    }
    dense(n.ws, n.bs, 1, n.w, a.h[7].data(), &a.zs);
    a.sigma = relu(a.zs);
    a.zf.assign(n.w, 0.0); a.f.assign(n.w, 0.0);
    dense(n.Wf, n.bf, n.w, n.w, a.h[7].data(), a.zf.data());
    for (int i = 0; i < n.w; ++i) a.f[i] = ORC_PLANT == 27 ? a.zf[i] : relu(a.zf[i]);
    a.in10 = a.f; a.in10.insert(a.in10.end(), a.gd.begin(), a.gd.end());
    if (ORC_PLANT == 29) for (int i = n.w; i < n.w + n.dd; ++i) a.in10[i] = 0.0;
    a.z10.assign(n.c, 0.0); a.h10.assign(n.c, 0.0);
    dense(n.W10, n.b10, n.c, n.w + n.dd, a.in10.data(), a.z10.data());
    for (int i = 0; i < n.c; ++i) a.h10[i] = ORC_PLANT == 28 ? a.z10[i] : relu(a.z10[i]);
    dense(n.W11, n.b11, 3, n.c, a.h10.data(), a.z11);
    for (int k = 0; k < 3; ++k) a.rgb[k] = sigmoid(a.z11[k]);
}
void global_backward(const GlobalNet& n, const GlobalAct& a, double dsigma, const double drgb[3], const GlobalNet& g) {
    double dz11[3];
    for (int k = 0; k < 3; ++k) dz11[k] = drgb[k] * a.rgb[k] * (1.0 - a.rgb[k]);
    std::vector<double> dh10(n.c), dz10(n.c), din10(n.w + n.dd), dh8(n.w, 0.0), dzf(n.w), tmp(n.w + n.dx);
    dense_backward(n.W11, 3, n.c, a.h10.data(), dz11, (double*)g.W11, (double*)g.b11, dh10.data());
    for (int i = 0; i < n.c; ++i) dz10[i] = (ORC_PLANT == 28 || a.z10[i] > 0.0) ? dh10[i] : 0.0;
    dense_backward(n.W10, n.c, n.w + n.dd, a.in10.data(), dz10.data(), (double*)g.W10, (double*)g.b10, din10.data());
    for (int i = 0; i < n.w; ++i) dzf[i] = (ORC_PLANT == 27 || a.zf[i] > 0.0) ? din10[i] : 0.0;
    dense_backward(n.Wf, n.w, n.w, a.h[7].data(), dzf.data(), (double*)g.Wf, (double*)g.bf, tmp.data());
    for (int i = 0; i < n.w; ++i) dh8[i] += tmp[i];
    double dzs = a.zs > 0.0 ? dsigma : 0.0;
    dense_backward(n.ws, 1, n.w, a.h[7].data(), &dzs, (double*)g.ws, (double*)g.bs, tmp.data());
    for (int i = 0; i < n.w; ++i) dh8[i] += tmp[i];
    std::vector<double> dh = dh8, dz(n.w);
    for (int k = 7; k >= 0; --k) {
        for (int i = 0; i < n.w; ++i) dz[i] = (k == 7) ? dh[i] : (a.z[k][i] > 0.0 ? dh[i] : 0.0);
        int in = (int)a.in[k].size();
        std::vector<double> din(in);
        dense_backward(n.W[k], n.w, in, a.in[k].data(), dz.data(), (double*)g.W[k], (double*)g.b[k],
                       k > 0 ? din.data() : nullptr);
        if (k > 0) for (int i = 0; i < n.w; ++i) dh[i] = din[i];   // the skip's gx part has no parameters upstream
    }
}

}  // namespace

extern "C" {

// ---- Eq.2/Eq.3 ------------------------------------------------------------
void orc_equirect_lut(int W, int H, float* sphi, float* cphi, float* sth, float* cth) {
    for (int u = 0; u < W; ++u) {
        float a, b, c, d;
        equirect_trig(W, H, u, 0, &a, &b, &c, &d);
        sphi[u] = a; cphi[u] = b;
    }
    for (int v = 0; v < H; ++v) {
        float a, b, c, d;
        equirect_trig(W, H, 0, v, &a, &b, &c, &d);
        sth[v] = c; cth[v] = d;
    }
}

// Rays for the given pixels (linear index v * W + u) of an equirect camera;
// pix == nullptr means all W*H pixels in raster order. o, d are [3][N].
void orc_equirect_rays(int W, int H, const float* c2w, const int64_t* pix, int64_t N, float* o, float* d) {
    for (int64_t r = 0; r < N; ++r) {
        int64_t p = pix ? pix[r] : r;
        int u = (int)(p % W), v = (int)(p / W);
        float sphi, cphi, sth, cth;
        equirect_trig(W, H, u, v, &sphi, &cphi, &sth, &cth);
        float dc[3] = {cth * sphi, ORC_PLANT == 11 ? sth : -sth, cth * cphi};
        float oo[3], dd[3];
        to_world(c2w, dc, oo, dd);
        for (int a = 0; a < 3; ++a) { o[a * N + r] = oo[a]; d[a * N + r] = dd[a]; }
    }
}

// Omni-directional stereo (the stereoscopic mode of Sec. 5 for panoramas):
// the ray of pixel (u, v) keeps its equirect direction but starts on the
// viewing circle of radius |eye| around the camera centre, at the point
// perpendicular to its horizontal heading: in the camera frame the origin
// offset is (eye cos(phi), 0, -eye sin(phi)) (eye > 0: the right eye, which
// sits at +x when looking along +z), rotated to the world as
//   o_i = t_i + fma(R_i2, oz, fma(R_i1, oy, R_i0 * ox)).
// eye = 0 gives the equirect rays exactly.
void orc_ods_rays(int W, int H, const float* c2w, float eye, const int64_t* pix, int64_t N, float* o, float* d) {
    for (int64_t r = 0; r < N; ++r) {
        int64_t p = pix ? pix[r] : r;
        int u = (int)(p % W), v = (int)(p / W);
        float sphi, cphi, sth, cth;
        equirect_trig(W, H, u, v, &sphi, &cphi, &sth, &cth);
        float dc[3] = {cth * sphi, -sth, cth * cphi};
        float oc[3] = {ORC_PLANT == 24 ? eye * sphi : eye * cphi, 0.0f, ORC_PLANT == 24 ? eye * cphi : -(eye * sphi)};
        float oo[3], dd[3];
        to_world(c2w, dc, oo, dd);
        for (int a = 0; a < 3; ++a) {
            const float* R = c2w + 4 * a;
            if (eye != 0.0f) oo[a] = R[3] + std::fma(R[2], oc[2], std::fma(R[1], oc[1], R[0] * oc[0]));
            o[a * N + r] = oo[a]; d[a * N + r] = dd[a];
        }
    }
}

// Pinhole rays (perspective viewports): x = ((u + 1/2) - W/2) / fx,
// y = ((v + 1/2) - H/2) / fy, z = 1, normalised with a correctly rounded
// sqrt of fma(x, x, fma(y, y, 1)); then to the world frame.
void orc_pinhole_rays(int W, int H, float fx, float fy, const float* c2w, int64_t N0, int64_t N, float* o, float* d) {
    for (int64_t r = 0; r < N; ++r) {
        int64_t p = N0 + r;
        int u = (int)(p % W), v = (int)(p / W);
        float x = ((float)u + 0.5f - 0.5f * (float)W) / fx;
        float y = ((float)v + 0.5f - 0.5f * (float)H) / fy;
        float nrm = std::sqrt(std::fma(x, x, std::fma(y, y, 1.0f)));
        float dc[3] = {x / nrm, y / nrm, 1.0f / nrm};
        float oo[3], dd[3];
        to_world(c2w, dc, oo, dd);
        for (int a = 0; a < 3; ++a) { o[a * N + r] = oo[a]; d[a * N + r] = dd[a]; }
    }
}

// ---- sampling -------------------------------------------------------------
// Per-ray sample counts (counts[N]).
void orc_count_samples(const OrcScene* s, int64_t N, const float* o, const float* d, int32_t* counts, int nthreads) {
    parallel_for(N, nthreads, [&](int64_t b, int64_t e, int) {
        std::vector<Seg> segs(s->max_samples);
        for (int64_t r = b; r < e; ++r) {
            float oo[3] = {o[r], o[N + r], o[2 * N + r]}, dd[3] = {d[r], d[N + r], d[2 * N + r]};
            counts[r] = sample_ray(*s, oo, dd, segs.data());
        }
    });
}

// Sample lists in ray-major order at the given exclusive offsets.
void orc_sample_rays(const OrcScene* s, int64_t N, const float* o, const float* d, const int64_t* offsets,
                     float* t_mid, float* delta, int32_t* ray_id, int32_t* voxel, int32_t* field, int nthreads) {
    parallel_for(N, nthreads, [&](int64_t b, int64_t e, int) {
        std::vector<Seg> segs(s->max_samples);
        for (int64_t r = b; r < e; ++r) {
            float oo[3] = {o[r], o[N + r], o[2 * N + r]}, dd[3] = {d[r], d[N + r], d[2 * N + r]};
            int n = sample_ray(*s, oo, dd, segs.data());
            for (int k = 0; k < n; ++k) {
                int64_t j = offsets[r] + k;
                t_mid[j] = segs[k].t_mid; delta[j] = segs[k].delta;
                ray_id[j] = (int32_t)r; voxel[j] = segs[k].voxel; field[j] = segs[k].field;
            }
        }
    });
}

// ---- per-field encoding frames ----------------------------------------------
// Axis-aligned box of the voxels labelled f in field_map: per axis the
// smallest and largest voxel index, box_lo = fma(imin, voxel, lo), box_hi =
// fma(imax + 1, voxel, lo); centre (box_lo + box_hi) * 0.5, half extent the
// largest of (box_hi - box_lo) * 0.5 over the axes (FP32). A field with no
// voxel gets centre 0 and half extent 1. frames [F][4].
void orc_field_frames(const int32_t* n, const float* lo, float voxel, const int32_t* field_map, int32_t F,
                      float* frames) {
    std::vector<int> mn(3 * (size_t)F, std::numeric_limits<int>::max()), mx(3 * (size_t)F, -1);
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                const int f = field_map[x + (int64_t)n[0] * (y + (int64_t)n[1] * z)];
                if (f < 0 || f >= F) continue;
                const int idx[3] = {x, y, z};
                for (int a = 0; a < 3; ++a) {
                    mn[3 * f + a] = std::min(mn[3 * f + a], idx[a]);
                    mx[3 * f + a] = std::max(mx[3 * f + a], idx[a]);
                }
            }
    for (int f = 0; f < F; ++f) {
        if (mx[3 * f] < 0) {
            frames[4 * f] = frames[4 * f + 1] = frames[4 * f + 2] = 0.0f;
            frames[4 * f + 3] = 1.0f;
            continue;
        }
        float h = 0.0f;
        for (int a = 0; a < 3; ++a) {
            const float blo = std::fma((float)mn[3 * f + a], voxel, lo[a]);
            const float bhi = std::fma((float)(mx[3 * f + a] + 1), voxel, lo[a]);
            frames[4 * f + a] = (blo + bhi) * 0.5f;
            h = std::max(h, (bhi - blo) * 0.5f);
        }
        frames[4 * f + 3] = h;
    }
}

// ---- encoding / MLP / compositing building blocks (for pins) ---------------
void orc_encode(const double* x, int L, double* out) { encode(x, L, out); }

void orc_local_mlp(const float* w, int hidden, int Lx, int Ld, const double* xh, const double* dir,
                   double* sigma, double* rgb) {
    int dx = 3 + 6 * Lx, dd = 3 + 6 * Ld;
    std::vector<double> wd = widen(w, local_params(hidden, dx, dd));
    LocalNet n = local_view(wd.data(), hidden, dx, dd);
    LocalAct a;
    local_forward(n, xh, dir, Lx, Ld, a);
    *sigma = a.sigma;
    for (int c = 0; c < 3; ++c) rgb[c] = a.rgb[c];
}

void orc_composite(int n, const double* sigma, const double* rgb, const double* t_mid, const double* delta,
                   double* C, double* D, double* A, double* w) {
    composite(n, sigma, rgb, t_mid, delta, C, D, A, w);
}

void orc_composite_backward(int n, const double* sigma, const double* rgb, const double* delta, const double* g,
                            double* dsigma, double* drgb) {
    composite_backward(n, sigma, rgb, delta, g, dsigma, drgb);
}

// ---- full render: sampling -> encoding -> local MLP -> compositing --------
// Per ray: rgb [3][N], depth [N], opacity [N]; optional per-sample sigma/rgb
// in ray-major order at `offsets` (may be null).
void orc_render_rays(const OrcScene* s, int64_t N, const float* o, const float* d, double* rgb, double* depth,
                     double* opacity, int nthreads) {
    const int dx = 3 + 6 * s->L_xyz, dd = 3 + 6 * s->L_dir;
    const size_t P = local_params(s->hidden, dx, dd);
    std::vector<double> wd = widen(s->weights, P * s->n_fields);
    parallel_for(N, nthreads, [&](int64_t b, int64_t e, int) {
        std::vector<Seg> segs(s->max_samples);
        std::vector<double> sig(s->max_samples), col(3 * s->max_samples), tm(s->max_samples), de(s->max_samples);
        LocalAct a;
        for (int64_t r = b; r < e; ++r) {
            float oo[3] = {o[r], o[N + r], o[2 * N + r]}, dv[3] = {d[r], d[N + r], d[2 * N + r]};
            int n = sample_ray(*s, oo, dv, segs.data());
            double dir[3] = {dv[0], dv[1], dv[2]};
            for (int k = 0; k < n; ++k) {
                double xh[3];
                sample_position(*s, oo, dv, segs[k].t_mid, segs[k].field, xh);
                LocalNet net = local_view(wd.data() + P * segs[k].field, s->hidden, dx, dd);
                local_forward(net, xh, dir, s->L_xyz, s->L_dir, a);
                sig[k] = a.sigma;
                for (int c = 0; c < 3; ++c) col[3 * k + c] = a.rgb[c];
                tm[k] = segs[k].t_mid; de[k] = segs[k].delta;
            }
            double C[3], D, A;
            composite(n, sig.data(), col.data(), tm.data(), de.data(), C, &D, &A, nullptr);
            for (int c = 0; c < 3; ++c) rgb[c * N + r] = C[c];
            depth[r] = D; opacity[r] = A;
        }
    });
}

// Per-sample network outputs in ray-major order (offsets as from the counts).
void orc_sample_outputs(const OrcScene* s, int64_t N, const float* o, const float* d, const int64_t* offsets,
                        double* sigma, double* rgb /*[3][S]*/, int64_t S, int nthreads) {
    const int dx = 3 + 6 * s->L_xyz, dd = 3 + 6 * s->L_dir;
    const size_t P = local_params(s->hidden, dx, dd);
    std::vector<double> wd = widen(s->weights, P * s->n_fields);
    parallel_for(N, nthreads, [&](int64_t b, int64_t e, int) {
        std::vector<Seg> segs(s->max_samples);
        LocalAct a;
        for (int64_t r = b; r < e; ++r) {
            float oo[3] = {o[r], o[N + r], o[2 * N + r]}, dv[3] = {d[r], d[N + r], d[2 * N + r]};
            int n = sample_ray(*s, oo, dv, segs.data());
            double dir[3] = {dv[0], dv[1], dv[2]};
            for (int k = 0; k < n; ++k) {
                double xh[3];
                sample_position(*s, oo, dv, segs[k].t_mid, segs[k].field, xh);
                LocalNet net = local_view(wd.data() + P * segs[k].field, s->hidden, dx, dd);
                local_forward(net, xh, dir, s->L_xyz, s->L_dir, a);
                int64_t j = offsets[r] + k;
                sigma[j] = a.sigma;
                for (int c = 0; c < 3; ++c) rgb[c * S + j] = a.rgb[c];
            }
        }
    });
}

// ---- training: L = 1/(3B) sum_rays sum_ch (C - C*)^2, gradient w.r.t. all
// local-field weights (Sec. 4.2 fine-tuning with an L2 photometric loss).
// grad is [n_fields][P] FP64 (overwritten). Returns the loss.
// grad_mag (optional, [n_fields][P]) receives the magnitude of each gradient
// entry (local_magnitude, composite_magnitude; dL/dC at the magnitude
// 2 (|C| + |C*|) / (3B) of its difference), for error bounds of other
// implementations: a rounding of relative size u in every term of an entry
// moves it by at most u times its magnitude. grad_kink (optional, with
// grad_mag) receives the magnitude of the terms through ReLU units whose
// pre-activation lies within tau of zero (see local_magnitude).
double orc_train_grad(const OrcScene* s, int64_t N, const float* o, const float* d, const float* target /*[3][N]*/,
                      double* grad, double* rgb_out /*[3][N] or null*/, int nthreads, double* grad_mag,
                      double tau, double* grad_kink) {
    const int dx = 3 + 6 * s->L_xyz, dd = 3 + 6 * s->L_dir;
    const size_t P = local_params(s->hidden, dx, dd);
    const size_t GP = P * s->n_fields;
    std::vector<double> wd = widen(s->weights, GP);
    int nt = std::max(1, nthreads);
    std::vector<std::vector<double>> gth(nt, std::vector<double>(GP, 0.0));
    std::vector<std::vector<double>> mth(grad_mag ? nt : 0, std::vector<double>(GP, 0.0));
    std::vector<std::vector<double>> kth(grad_mag && grad_kink ? nt : 0, std::vector<double>(GP, 0.0));
    std::vector<double> lth(nt, 0.0);
    parallel_for(N, nt, [&](int64_t b, int64_t e, int t) {
        std::vector<Seg> segs(s->max_samples);
        std::vector<LocalAct> acts(s->max_samples);
        std::vector<double> sig(s->max_samples), col(3 * s->max_samples), tm(s->max_samples), de(s->max_samples);
        std::vector<double> dsig(s->max_samples), dcol(3 * s->max_samples);
        std::vector<double> msig(s->max_samples), mcol(3 * s->max_samples);
        for (int64_t r = b; r < e; ++r) {
            float oo[3] = {o[r], o[N + r], o[2 * N + r]}, dv[3] = {d[r], d[N + r], d[2 * N + r]};
            int n = sample_ray(*s, oo, dv, segs.data());
            double dir[3] = {dv[0], dv[1], dv[2]};
            for (int k = 0; k < n; ++k) {
                double xh[3];
                sample_position(*s, oo, dv, segs[k].t_mid, segs[k].field, xh);
                LocalNet net = local_view(wd.data() + P * segs[k].field, s->hidden, dx, dd);
                local_forward(net, xh, dir, s->L_xyz, s->L_dir, acts[k]);
                sig[k] = acts[k].sigma;
                for (int c = 0; c < 3; ++c) col[3 * k + c] = acts[k].rgb[c];
                tm[k] = segs[k].t_mid; de[k] = segs[k].delta;
            }
            double C[3], D, A;
            composite(n, sig.data(), col.data(), tm.data(), de.data(), C, &D, &A, nullptr);
            double g[3];
            for (int c = 0; c < 3; ++c) {
                double diff = C[c] - (double)target[c * N + r];
                lth[t] += diff * diff / (3.0 * N);
                g[c] = 2.0 * diff / (3.0 * N);
                if (rgb_out) rgb_out[c * N + r] = C[c];
            }
            composite_backward(n, sig.data(), col.data(), de.data(), g, dsig.data(), dcol.data());
            for (int k = 0; k < n; ++k) {
                LocalNet net = local_view(wd.data() + P * segs[k].field, s->hidden, dx, dd);
                LocalNet gn = local_view(gth[t].data() + P * segs[k].field, s->hidden, dx, dd);
                local_backward(net, acts[k], dsig[k], &dcol[3 * k], gn);
            }
            if (grad_mag) {
                double gm[3];
                for (int c = 0; c < 3; ++c)
                    gm[c] = 2.0 * (std::fabs(C[c]) + std::fabs((double)target[c * N + r])) / (3.0 * N);
                composite_magnitude(n, sig.data(), col.data(), de.data(), gm, msig.data(), mcol.data());
                for (int k = 0; k < n; ++k) {
                    LocalNet net = local_view(wd.data() + P * segs[k].field, s->hidden, dx, dd);
                    LocalNet gmv = local_view(mth[t].data() + P * segs[k].field, s->hidden, dx, dd);
                    LocalNet gkv;
                    if (grad_kink) gkv = local_view(kth[t].data() + P * segs[k].field, s->hidden, dx, dd);
                    local_magnitude(net, acts[k], msig[k], &mcol[3 * k], gmv, tau, grad_kink ? &gkv : nullptr);
                }
            }
        }
    });
    double loss = 0.0;
    for (size_t i = 0; i < GP; ++i) grad[i] = 0.0;
    for (int t = 0; t < nt; ++t) {
        loss += lth[t];
        for (size_t i = 0; i < GP; ++i) grad[i] += gth[t][i];
    }
    if (grad_mag) {
        for (size_t i = 0; i < GP; ++i) grad_mag[i] = 0.0;
        for (int t = 0; t < nt; ++t)
            for (size_t i = 0; i < GP; ++i) grad_mag[i] += mth[t][i];
    }
    if (grad_mag && grad_kink) {
        for (size_t i = 0; i < GP; ++i) grad_kink[i] = 0.0;
        for (int t = 0; t < nt; ++t)
            for (size_t i = 0; i < GP; ++i) grad_kink[i] += kth[t][i];
    }
    return loss;
}

// ---- distillation (Sec. 4.2, Eq.7): each local field is fitted to the global
// field at points inside its own region. With point i (position x_i, view
// direction d_i) owned by field k(i), local outputs sigma^k_i, c^k_i and the
// global field's targets sigma_i, c_i:
//   L = sum_k (1/I_k) sum_{i of field k} [(sigma^k_i - sigma_i)^2 + |c^k_i - c_i|^2],
// I_k the number of points of field k (points with a field id outside
// [0, n_fields) are ignored). The local field sees the point through the
// renderer's own sample position with t = 0: p = fma(0, d, x) = x. Returns
// L; grad [n_fields][P] (FP64, overwritten); sigma/rgb outputs optional.
double orc_distill(const OrcScene* s, int64_t M, const float* x, const float* dir, const int32_t* field,
                   const float* tsig, const float* trgb /*[3][M]*/, double* grad, double* sig_out,
                   double* rgb_out /*[3][M]*/, int nthreads) {
    const int dx = 3 + 6 * s->L_xyz, dd = 3 + 6 * s->L_dir;
    const size_t P = local_params(s->hidden, dx, dd);
    const size_t GP = P * s->n_fields;
    std::vector<double> wd = widen(s->weights, GP);
    std::vector<int64_t> I(s->n_fields, 0);
    for (int64_t i = 0; i < M; ++i)
        if (field[i] >= 0 && field[i] < s->n_fields) ++I[field[i]];
    int nt = std::max(1, nthreads);
    std::vector<std::vector<double>> gth(nt, std::vector<double>(GP, 0.0));
    std::vector<double> lth(nt, 0.0);
    parallel_for(M, nt, [&](int64_t b, int64_t e, int t) {
        LocalAct a;
        for (int64_t i = b; i < e; ++i) {
            const int k = field[i];
            if (k < 0 || k >= s->n_fields) continue;
            float oo[3] = {x[i], x[M + i], x[2 * M + i]}, dv[3] = {dir[i], dir[M + i], dir[2 * M + i]};
            double xh[3], dd3[3] = {dv[0], dv[1], dv[2]};
            sample_position(*s, oo, dv, 0.0f, k, xh);
            LocalNet net = local_view(wd.data() + P * k, s->hidden, dx, dd);
            local_forward(net, xh, dd3, s->L_xyz, s->L_dir, a);
            const double inv = ORC_PLANT == 21 ? 1.0 / (double)M : 1.0 / (double)I[k];
            const double ds = a.sigma - (double)tsig[i];
            double dsig = 2.0 * ds * inv, drgb[3];
            double l = ds * ds;
            for (int c = 0; c < 3; ++c) {
                const double dc = a.rgb[c] - (double)trgb[c * M + i];
                l += dc * dc;
                drgb[c] = 2.0 * dc * inv;
            }
            if (ORC_PLANT == 22) dsig = 0.0;
            lth[t] += l * inv;
            LocalNet gn = local_view(gth[t].data() + P * k, s->hidden, dx, dd);
            local_backward(net, a, dsig, drgb, gn);
            if (sig_out) sig_out[i] = a.sigma;
            if (rgb_out) for (int c = 0; c < 3; ++c) rgb_out[c * M + i] = a.rgb[c];
        }
    });
    double loss = 0.0;
    for (size_t q = 0; q < GP; ++q) grad[q] = 0.0;
    for (int t = 0; t < nt; ++t) {
        loss += lth[t];
        for (size_t q = 0; q < GP; ++q) grad[q] += gth[t][q];
    }
    return loss;
}

// ---- global omnidirectional field ----------------------------------------
// Sample placement uniform in inverse depth over [near, far] (Sec. 3.2
// places the global field's samples evenly in inverse distance), FP32 spec:
//   a = 1/near, b = 1/far, s_i = i / (N - 1), t_i = 1 / fma(s_i, b, (1 - s_i) a),
// which gives 1/near and 1/far exactly at the two ends;
//   delta_i = t_{i+1} - t_i, and delta_{N-1} = 0.
void orc_invdepth_t(int n_samples, float near_, float far_, float* t, float* delta) {
    float a = 1.0f / near_, b = 1.0f / far_;
    for (int i = 0; i < n_samples; ++i) {
        float si = (float)i / (float)(n_samples - 1);
        t[i] = 1.0f / std::fma(si, b, (1.0f - si) * a);
    }
    for (int i = 0; i < n_samples; ++i) delta[i] = (i + 1 < n_samples) ? t[i + 1] - t[i] : 0.0f;
}

struct OrcGlobal {
    int32_t width, color_width, L_xyz, L_dir, n_samples;
    float near_, far_;
    float center[3];
    float half_extent;
    const float* weights;
    // occupancy grid for the density max: grid[n2][n1][n0]
    int32_t n[3];
    float lo[3];
    float voxel;
};

// Forward + backward of the global field over N rays; returns the loss and
// writes the gradient [P] (FP64), per-ray colour [3][N], depth, opacity, and
// the per-voxel max of sample density into occ_max (FP64, initialised by the
// caller).
double orc_global_step(const OrcGlobal* g, int64_t N, const float* o, const float* d, const float* target,
                       double* grad, double* rgb_out, double* depth_out, double* opacity_out,
                       double* occ_max, int nthreads) {
    const int dx = 3 + 6 * g->L_xyz, dd = 3 + 6 * g->L_dir, ns = g->n_samples;
    const size_t P = global_params(g->width, g->color_width, dx, dd);
    std::vector<double> wd = widen(g->weights, P);
    GlobalNet net = global_view(wd.data(), g->width, g->color_width, dx, dd);
    std::vector<float> tt(ns), dl(ns);
    orc_invdepth_t(ns, g->near_, g->far_, tt.data(), dl.data());
    int nt = std::max(1, nthreads);
    std::vector<std::vector<double>> gth(nt, std::vector<double>(P, 0.0));
    std::vector<double> lth(nt, 0.0);
    const size_t ncell = (size_t)g->n[0] * g->n[1] * g->n[2];
    std::vector<std::vector<double>> occ_th(nt, std::vector<double>(occ_max ? ncell : 0, 0.0));
    const float inv_h = 1.0f / g->half_extent, inv_vox = 1.0f / g->voxel;
    parallel_for(N, nt, [&](int64_t b, int64_t e, int t) {
        std::vector<GlobalAct> acts(ns);
        std::vector<double> sig(ns), col(3 * ns), tm(ns), de(ns), dsig(ns), dcol(3 * ns);
        GlobalNet gn = global_view(gth[t].data(), g->width, g->color_width, dx, dd);
        for (int64_t r = b; r < e; ++r) {
            float oo[3] = {o[r], o[N + r], o[2 * N + r]}, dv[3] = {d[r], d[N + r], d[2 * N + r]};
            double dir[3] = {dv[0], dv[1], dv[2]};
            for (int k = 0; k < ns; ++k) {
                double xh[3];
                int cell[3];
                bool inside = true;
                for (int a = 0; a < 3; ++a) {
                    float p = std::fma(tt[k], dv[a], oo[a]);
                    xh[a] = (double)((p - g->center[a]) * inv_h);
                    float q = (p - g->lo[a]) * inv_vox;
                    inside = inside && (q >= 0.0f) && (q < (float)g->n[a]);
                    cell[a] = inside ? (int)std::floor(q) : 0;
                }
                global_forward(net, xh, dir, g->L_xyz, g->L_dir, acts[k]);
                sig[k] = acts[k].sigma;
                for (int c = 0; c < 3; ++c) col[3 * k + c] = acts[k].rgb[c];
                tm[k] = tt[k]; de[k] = dl[k];
                if (occ_max && inside) {
                    size_t lin = cell[0] + (size_t)g->n[0] * (cell[1] + (size_t)g->n[1] * cell[2]);
                    occ_th[t][lin] = std::max(occ_th[t][lin], sig[k]);
                }
            }
            double C[3], D, A;
            composite(ns, sig.data(), col.data(), tm.data(), de.data(), C, &D, &A, nullptr);
            if (rgb_out) for (int c = 0; c < 3; ++c) rgb_out[c * N + r] = C[c];
            if (depth_out) depth_out[r] = D;
            if (opacity_out) opacity_out[r] = A;
            double gC[3];
            for (int c = 0; c < 3; ++c) {
                double diff = C[c] - (double)target[c * N + r];
                lth[t] += diff * diff / (3.0 * N);
                gC[c] = 2.0 * diff / (3.0 * N);
            }
            composite_backward(ns, sig.data(), col.data(), de.data(), gC, dsig.data(), dcol.data());
            for (int k = 0; k < ns; ++k) global_backward(net, acts[k], dsig[k], &dcol[3 * k], gn);
        }
    });
    double loss = 0.0;
    for (size_t i = 0; i < P; ++i) grad[i] = 0.0;
    for (int t = 0; t < nt; ++t) {
        loss += lth[t];
        for (size_t i = 0; i < P; ++i) grad[i] += gth[t][i];
        if (occ_max) for (size_t i = 0; i < ncell; ++i) occ_max[i] = std::max(occ_max[i], occ_th[t][i]);
    }
    return loss;
}

// The distillation targets: the global field's density and colour at given
// points (position x, direction d): the global step's sample position with
// t = 0, xhat = (fma(0, d, x) - center) / half_extent, FP64 network.
void orc_global_points(const OrcGlobal* g, int64_t M, const float* x, const float* dir, double* sig,
                       double* rgb /*[3][M]*/, int nthreads) {
    const int dx = 3 + 6 * g->L_xyz, dd = 3 + 6 * g->L_dir;
    const size_t P = global_params(g->width, g->color_width, dx, dd);
    std::vector<double> wd = widen(g->weights, P);
    GlobalNet net = global_view(wd.data(), g->width, g->color_width, dx, dd);
    const float inv_h = 1.0f / g->half_extent;
    parallel_for(M, std::max(1, nthreads), [&](int64_t b, int64_t e, int) {
        GlobalAct a;
        for (int64_t i = b; i < e; ++i) {
            float dv[3] = {dir[i], dir[M + i], dir[2 * M + i]};
            double xh[3], d3[3] = {dv[0], dv[1], dv[2]};
            for (int c = 0; c < 3; ++c)
                xh[c] = (double)((std::fma(0.0f, dv[c], x[c * M + i]) - g->center[c]) * inv_h);
            global_forward(net, xh, d3, g->L_xyz, g->L_dir, a);
            sig[i] = a.sigma;
            for (int c = 0; c < 3; ++c) rgb[c * M + i] = a.rgb[c];
        }
    });
}

// Global field forward at explicit points (pins and per-sample checks).
void orc_global_mlp(const float* w, int width, int color_width, int Lx, int Ld, const double* xh, const double* dir,
                    double* sigma, double* rgb) {
    int dx = 3 + 6 * Lx, dd = 3 + 6 * Ld;
    std::vector<double> wd = widen(w, global_params(width, color_width, dx, dd));
    GlobalNet n = global_view(wd.data(), width, color_width, dx, dd);
    GlobalAct a;
    global_forward(n, xh, dir, Lx, Ld, a);
    *sigma = a.sigma;
    for (int c = 0; c < 3; ++c) rgb[c] = a.rgb[c];
}

int64_t orc_local_params(int hidden, int Lx, int Ld) { return (int64_t)local_params(hidden, 3 + 6 * Lx, 3 + 6 * Ld); }
int64_t orc_global_params(int width, int color_width, int Lx, int Ld) {
    return (int64_t)global_params(width, color_width, 3 + 6 * Lx, 3 + 6 * Ld);
}

// ---- Stage I occupancy (Sec. 4.1, Alg.1) -----------------------------------
// Per-ray measurement from dense samples [N][S] (FP32 inputs, FP64 result).
void orc_depth_stats(int64_t N, int S, const float* t, const float* delta, const float* sigma, double* D, double* U,
                     double* A) {
    std::vector<double> sg(S), tt(S), dl(S);
    for (int64_t r = 0; r < N; ++r) {
        for (int k = 0; k < S; ++k) {
            sg[k] = sigma[r * S + k]; tt[k] = t[r * S + k]; dl[k] = delta[r * S + k];
        }
        depth_stats(S, sg.data(), tt.data(), dl.data(), &D[r], &U[r], &A[r]);
    }
}

// One pose's update of the logit grid [n2][n1][n0] (in place) from N rays.
void orc_occupancy_update(const OrcOcc* g, float* logit, float* prob, int64_t N, const float* o, const float* d,
                          const float* depth, const float* uncert, const float* opacity, int nthreads) {
    const size_t ncell = (size_t)g->n[0] * g->n[1] * g->n[2];
    const float inv_vox = 1.0f / g->voxel;
    int nt = std::max(1, nthreads);
    std::vector<std::vector<float>> hit(nt, std::vector<float>(ncell, 0.0f));
    std::vector<std::vector<uint8_t>> miss(nt, std::vector<uint8_t>(ncell, 0));
    parallel_for(N, nt, [&](int64_t b, int64_t e, int th) {
        for (int64_t r = b; r < e; ++r) {
            const float Dr = depth[r], Ur = uncert[r], Ar = opacity[r];
            if (!(Ar >= g->min_opacity) || !std::isfinite(Dr) || !std::isfinite(Ur) || !(Ur >= 0.0f)) continue;
            const float oo[3] = {o[r], o[N + r], o[2 * N + r]}, dv[3] = {d[r], d[N + r], d[2 * N + r]};
            bool bad = false;
            for (int a = 0; a < 3; ++a) bad = bad || !(oo[a] == oo[a]) || !(dv[a] == dv[a]);
            if (bad) continue;
            const float edge = ORC_PLANT == 14 ? Dr : Dr - Ur;
            const float h = ORC_PLANT == 17 ? g->l_hit : g->l_hit / (1.0f + Ur * inv_vox);
            walk_ray(g->n, g->lo, g->voxel, g->near_, g->far_, oo, dv, [&](int64_t lin, float t_in, float t_out) {
                if (t_out <= edge) { miss[th][lin] = 1; return true; }
                if (Dr < t_out) {
                    if (t_in <= Dr) hit[th][lin] = std::max(hit[th][lin], h);
                    return false;
                }
                return true;
            });
        }
    });
    for (size_t v = 0; v < ncell; ++v) {
        float hv = 0.0f;
        bool mv = false;
        for (int t = 0; t < nt; ++t) { hv = std::max(hv, hit[t][v]); mv = mv || miss[t][v]; }
        float l = logit[v];
        const bool use_hit = ORC_PLANT == 15 ? (hv > 0.0f && !mv) : hv > 0.0f;
        if (use_hit || mv) {
            l = use_hit ? l + hv : l + g->l_miss;
            if (ORC_PLANT != 13) l = std::min(std::max(l, g->l_min), g->l_max);
            logit[v] = l;
        }
        if (prob) prob[v] = (float)(1.0 / (1.0 + std::exp(-(double)l)));
    }
}

// Stage I measurement by the global field: its forward over the inverse-depth
// samples of each ray, then the per-ray depth, uncertainty and opacity.
void orc_global_measure(const OrcGlobal* g, int64_t N, const float* o, const float* d, double* depth,
                        double* uncert, double* opacity, int nthreads) {
    const int dx = 3 + 6 * g->L_xyz, dd = 3 + 6 * g->L_dir, ns = g->n_samples;
    const size_t P = global_params(g->width, g->color_width, dx, dd);
    std::vector<double> wd = widen(g->weights, P);
    GlobalNet net = global_view(wd.data(), g->width, g->color_width, dx, dd);
    std::vector<float> tt(ns), dl(ns);
    orc_invdepth_t(ns, g->near_, g->far_, tt.data(), dl.data());
    const float inv_h = 1.0f / g->half_extent;
    parallel_for(N, std::max(1, nthreads), [&](int64_t b, int64_t e, int) {
        GlobalAct act;
        std::vector<double> sig(ns), tm(ns), de(ns);
        for (int64_t r = b; r < e; ++r) {
            float oo[3] = {o[r], o[N + r], o[2 * N + r]}, dv[3] = {d[r], d[N + r], d[2 * N + r]};
            double dir[3] = {dv[0], dv[1], dv[2]};
            for (int k = 0; k < ns; ++k) {
                double xh[3];
                for (int a = 0; a < 3; ++a) xh[a] = (double)((std::fma(tt[k], dv[a], oo[a]) - g->center[a]) * inv_h);
                global_forward(net, xh, dir, g->L_xyz, g->L_dir, act);
                sig[k] = act.sigma; tm[k] = tt[k]; de[k] = dl[k];
            }
            depth_stats(ns, sig.data(), tm.data(), de.data(), &depth[r], &uncert[r], &opacity[r]);
        }
    });
}

// ---- Stage II of Alg.1 (Sec. 4.2): adaptive field assignment ---------------
// S voxels are occupied (occ > thr); field k (0-based, k < n) receives
// s_k = floor(S / n) + (k < S mod n ? 1 : 0) of them, so sizes differ by at
// most one. For k = 0, 1, ...: the anchor is the unassigned occupied voxel of
// smallest linear index (the minimum coordinate, z then y then x); the field
// takes the s_k unassigned occupied voxels nearest to the anchor by squared
// Euclidean distance between voxel indices, ties to the smaller linear index
// (the anchor itself, at distance 0, first). Unoccupied voxels get -1.
// Returns S.
int64_t orc_assign_fields(const int32_t* n, const float* occ, float thr, int32_t n_fields, int32_t* field_map) {
    const int64_t nvox = (int64_t)n[0] * n[1] * n[2];
    std::vector<int64_t> occl;
    for (int64_t v = 0; v < nvox; ++v) {
        field_map[v] = -1;
        if (occ[v] > thr) occl.push_back(v);
    }
    const int64_t S = (int64_t)occl.size();
    if (n_fields < 1) return S;
    const int64_t base = S / n_fields, rem = S % n_fields;
    std::vector<char> done(S, 0);
    struct Cand { int64_t d2, lin, i; };
    std::vector<Cand> cand;
    for (int32_t k = 0; k < n_fields; ++k) {
        const int64_t sk = ORC_PLANT == 20 ? (k + 1 < n_fields ? base : S - base * (n_fields - 1))
                                           : base + (k < rem ? 1 : 0);
        if (sk == 0) continue;
        int64_t a = -1;
        for (int64_t i = 0; i < S; ++i)
            if (!done[i] && (a < 0 || ORC_PLANT == 18)) a = i;   // smallest index (plant: largest)
        const int64_t al = occl[a];
        const int64_t ax = al % n[0], ay = (al / n[0]) % n[1], az = al / ((int64_t)n[0] * n[1]);
        cand.clear();
        for (int64_t i = 0; i < S; ++i) {
            if (done[i]) continue;
            const int64_t l = occl[i];
            const int64_t dx = l % n[0] - ax, dy = (l / n[0]) % n[1] - ay, dz = l / ((int64_t)n[0] * n[1]) - az;
            const int64_t d2 = ORC_PLANT == 19 ? std::llabs(dx) + std::llabs(dy) + std::llabs(dz)
                                               : dx * dx + dy * dy + dz * dz;
            cand.push_back({d2, l, i});
        }
        const int64_t take = std::min<int64_t>(sk, (int64_t)cand.size());
        std::partial_sort(cand.begin(), cand.begin() + take, cand.end(), [](const Cand& x, const Cand& y) {
            return x.d2 != y.d2 ? x.d2 < y.d2 : x.lin < y.lin;
        });
        for (int64_t j = 0; j < take; ++j) {
            field_map[cand[j].lin] = k;
            done[cand[j].i] = 1;
        }
    }
    return S;
}

// The uniform decomposition (the 360Roam-u variant of Sec. 6): b[a] blocks
// per axis, voxel index i in block floor(i * b[a] / n[a]); the fields are the
// blocks that hold an occupied voxel, numbered in linear block order (x
// fastest). Returns the number of fields.
int32_t orc_assign_uniform(const int32_t* n, const float* occ, float thr, const int32_t* b, int32_t* field_map) {
    const int64_t nvox = (int64_t)n[0] * n[1] * n[2];
    const int64_t nb = (int64_t)b[0] * b[1] * b[2];
    std::vector<int64_t> blk(nvox);
    std::vector<int32_t> id(nb, -1);
    for (int64_t v = 0; v < nvox; ++v) {
        const int64_t x = v % n[0], y = (v / n[0]) % n[1], z = v / ((int64_t)n[0] * n[1]);
        blk[v] = x * b[0] / n[0] + b[0] * (y * b[1] / n[1] + b[1] * (z * b[2] / n[2]));
        if (occ[v] > thr) id[blk[v]] = 0;
    }
    int32_t count = 0;
    for (int64_t q = 0; q < nb; ++q)
        if (id[q] == 0) id[q] = count++;
    for (int64_t v = 0; v < nvox; ++v) field_map[v] = occ[v] > thr ? id[blk[v]] : -1;
    return count;
}

// ---- Adam (Sec. 6.1 training details: beta1 0.9, beta2 0.99) -------------
// m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), FP64.
void orc_adam(int64_t n, double* w, const double* g, double* m, double* v, int64_t step, double lr, double b1,
              double b2, double eps) {
    double c1 = 1.0 - std::pow(b1, (double)step), c2 = 1.0 - std::pow(b2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (std::sqrt(v[i] / c2) + eps);
    }
}

}  // extern "C"
