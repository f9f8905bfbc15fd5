// mf_device.hpp -- device building blocks for the MadFlow hot path on gfx950.
//
// Complex arithmetic, chiral-basis spinor algebra for the helicity
// amplitudes (Sec. 2.3: external wavefunctions, vertices, propagators),
// the counter-based Philox4x32-10 generator (Salmon et al., SC'11) and
// compensated (Neumaier / TwoSum) accumulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

template <typename T>
struct cplx {
    T x, y;
    __host__ __device__ __forceinline__ cplx() {}
    __host__ __device__ __forceinline__ cplx(T a, T b) : x(a), y(b) {}
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return cplx<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// Chiral representation: gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]],
// spinor components (L0, L1, R0, R1).  For a real 4-vector j:
//   j.sigma    = [[j0 - j3, -j1 + i j2], [-j1 - i j2, j0 + j3]]
//   j.sigmabar = [[j0 + j3,  j1 - i j2], [ j1 + i j2, j0 - j3]]
// ---------------------------------------------------------------------------

// s += a x gamma.(SGN j) for a row spinor a: (aR (j.sigmabar), aL (j.sigma)).
template <int SGN = 1, typename T>
__host__ __device__ __forceinline__ void rowslash_acc(const cplx<T>* a, const T* jin, cplx<T>& s0, cplx<T>& s1,
                                             cplx<T>& s2, cplx<T>& s3)
{
    const T j[4] = {(T)SGN * jin[0], (T)SGN * jin[1], (T)SGN * jin[2], (T)SGN * jin[3]};
    const T jp = j[0] + j[3], jm = j[0] - j[3];
    // s0 += aR0 (j0 + j3) + aR1 (j1 + i j2)
    s0.x += a[2].x * jp + a[3].x * j[1] - a[3].y * j[2];
    s0.y += a[2].y * jp + a[3].y * j[1] + a[3].x * j[2];
    // s1 += aR0 (j1 - i j2) + aR1 (j0 - j3)
    s1.x += a[2].x * j[1] + a[2].y * j[2] + a[3].x * jm;
    s1.y += a[2].y * j[1] - a[2].x * j[2] + a[3].y * jm;
    // s2 += aL0 (j0 - j3) + aL1 (-j1 - i j2)
    s2.x += a[0].x * jm - a[1].x * j[1] + a[1].y * j[2];
    s2.y += a[0].y * jm - a[1].y * j[1] - a[1].x * j[2];
    // s3 += aL0 (-j1 + i j2) + aL1 (j0 + j3)
    s3.x += -a[0].x * j[1] - a[0].y * j[2] + a[1].x * jp;
    s3.y += -a[0].y * j[1] + a[0].x * j[2] + a[1].y * jp;
}

// out = s x (K-slash + m) x (fr + i fi) for a row spinor s.
template <typename T>
__host__ __device__ __forceinline__ void rowprop(cplx<T> s0, cplx<T> s1, cplx<T> s2, cplx<T> s3, const T* K, T m,
                                        T fr, T fi, cplx<T>* out)
{
    const T kp = K[0] + K[3], km = K[0] - K[3];
    cplx<T> t0, t1, t2, t3;
    // t0 = m s0 + s2 (K0 + K3) + s3 (K1 + i K2)
    t0.x = m * s0.x + s2.x * kp + s3.x * K[1] - s3.y * K[2];
    t0.y = m * s0.y + s2.y * kp + s3.y * K[1] + s3.x * K[2];
    // t1 = m s1 + s2 (K1 - i K2) + s3 (K0 - K3)
    t1.x = m * s1.x + s2.x * K[1] + s2.y * K[2] + s3.x * km;
    t1.y = m * s1.y + s2.y * K[1] - s2.x * K[2] + s3.y * km;
    // t2 = s0 (K0 - K3) + s1 (-K1 - i K2) + m s2
    t2.x = s0.x * km - s1.x * K[1] + s1.y * K[2] + m * s2.x;
    t2.y = s0.y * km - s1.y * K[1] - s1.x * K[2] + m * s2.y;
    // t3 = s0 (-K1 + i K2) + s1 (K0 + K3) + m s3
    t3.x = -s0.x * K[1] - s0.y * K[2] + s1.x * kp + m * s3.x;
    t3.y = -s0.y * K[1] + s0.x * K[2] + s1.y * kp + m * s3.y;
    const cplx<T> f(fr, fi);
    out[0] = cmul(t0, f);
    out[1] = cmul(t1, f);
    out[2] = cmul(t2, f);
    out[3] = cmul(t3, f);
}

// out = (K-slash + m) w x (fr + i fi) for a column spinor w:
// ((m wL + (K.sigma) wR), ((K.sigmabar) wL + m wR)).
template <typename T>
__host__ __device__ __forceinline__ void colprop(const cplx<T>* w, const T* K, T m, T fr, T fi, cplx<T>* out)
{
    const T kp = K[0] + K[3], km = K[0] - K[3];
    cplx<T> t0, t1, t2, t3;
    // t0 = m w0 + (K0 - K3) w2 + (-K1 + i K2) w3
    t0.x = m * w[0].x + km * w[2].x - K[1] * w[3].x - K[2] * w[3].y;
    t0.y = m * w[0].y + km * w[2].y - K[1] * w[3].y + K[2] * w[3].x;
    // t1 = m w1 + (-K1 - i K2) w2 + (K0 + K3) w3
    t1.x = m * w[1].x - K[1] * w[2].x + K[2] * w[2].y + kp * w[3].x;
    t1.y = m * w[1].y - K[1] * w[2].y - K[2] * w[2].x + kp * w[3].y;
    // t2 = (K0 + K3) w0 + (K1 - i K2) w1 + m w2
    t2.x = kp * w[0].x + K[1] * w[1].x + K[2] * w[1].y + m * w[2].x;
    t2.y = kp * w[0].y + K[1] * w[1].y - K[2] * w[1].x + m * w[2].y;
    // t3 = (K1 + i K2) w0 + (K0 - K3) w1 + m w3
    t3.x = K[1] * w[0].x - K[2] * w[0].y + km * w[1].x + m * w[3].x;
    t3.y = K[1] * w[0].y + K[2] * w[0].x + km * w[1].y + m * w[3].y;
    const cplx<T> f(fr, fi);
    out[0] = cmul(t0, f);
    out[1] = cmul(t1, f);
    out[2] = cmul(t2, f);
    out[3] = cmul(t3, f);
}

// acc += gamma.(SGN e) w for a real 4-vector e and a complex column w.
template <int SGN = 1, typename T>
__host__ __device__ __forceinline__ void slashcol_acc(const T* ein, const cplx<T>* v, cplx<T>* W)
{
    const T e[4] = {(T)SGN * ein[0], (T)SGN * ein[1], (T)SGN * ein[2], (T)SGN * ein[3]};
    const T ep = e[0] + e[3], em = e[0] - e[3];
    W[0].x += em * v[2].x - e[1] * v[3].x - e[2] * v[3].y;
    W[0].y += em * v[2].y - e[1] * v[3].y + e[2] * v[3].x;
    W[1].x += -e[1] * v[2].x + e[2] * v[2].y + ep * v[3].x;
    W[1].y += -e[1] * v[2].y - e[2] * v[2].x + ep * v[3].y;
    W[2].x += ep * v[0].x + e[1] * v[1].x + e[2] * v[1].y;
    W[2].y += ep * v[0].y + e[1] * v[1].y - e[2] * v[1].x;
    W[3].x += e[1] * v[0].x - e[2] * v[0].y + em * v[1].x;
    W[3].y += e[1] * v[0].y + e[2] * v[0].x + em * v[1].y;
}

// Orders the LDS traffic of the lanes of one wavefront (no hardware barrier:
// a wavefront executes in lockstep; the fences keep the compiler and the
// memory model from reordering the accesses across this point).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// c^mu = a gamma^mu v = aL sigma^mu vR + aR sigmabar^mu vL.  The four
// components are sums and differences of four two-term products,
//   P = a0 v2 + a3 v1,  Q = a1 v3 + a2 v0,  R = a0 v3 - a2 v1,  S = a1 v2 - a3 v0:
//   c0 = P + Q,  c3 = P - Q,  c1 = R + S,  c2 = i (S - R).
template <typename T>
__host__ __device__ __forceinline__ void bilinear(const cplx<T>* a, const cplx<T>* v, cplx<T>* c)
{
    const T Px = a[0].x * v[2].x - a[0].y * v[2].y + a[3].x * v[1].x - a[3].y * v[1].y;
    const T Py = a[0].x * v[2].y + a[0].y * v[2].x + a[3].x * v[1].y + a[3].y * v[1].x;
    const T Qx = a[1].x * v[3].x - a[1].y * v[3].y + a[2].x * v[0].x - a[2].y * v[0].y;
    const T Qy = a[1].x * v[3].y + a[1].y * v[3].x + a[2].x * v[0].y + a[2].y * v[0].x;
    const T Rx = a[0].x * v[3].x - a[0].y * v[3].y - a[2].x * v[1].x + a[2].y * v[1].y;
    const T Ry = a[0].x * v[3].y + a[0].y * v[3].x - a[2].x * v[1].y - a[2].y * v[1].x;
    const T Sx = a[1].x * v[2].x - a[1].y * v[2].y - a[3].x * v[0].x + a[3].y * v[0].y;
    const T Sy = a[1].x * v[2].y + a[1].y * v[2].x - a[3].x * v[0].y - a[3].y * v[0].x;
    c[0] = cplx<T>(Px + Qx, Py + Qy);
    c[3] = cplx<T>(Px - Qx, Py - Qy);
    c[1] = cplx<T>(Rx + Sx, Ry + Sy);
    c[2] = cplx<T>(Ry - Sy, Sx - Rx);
}

// (ar, ai) += SGN c^mu j_mu for complex c and real j.
template <int SGN = 1, typename T>
__host__ __device__ __forceinline__ void cdotj(const cplx<T>* c, const T* j, T& ar, T& ai)
{
    const T r = c[0].x * j[0] - c[1].x * j[1] - c[2].x * j[2] - c[3].x * j[3];
    const T i = c[0].y * j[0] - c[1].y * j[1] - c[2].y * j[2] - c[3].y * j[3];
    ar += (T)SGN * r;
    ai += (T)SGN * i;
}

// A pointer into the object store, declared 16-byte aligned.
template <typename T>
__device__ __forceinline__ const T* al16(const T* p)
{
    return static_cast<const T*>(__builtin_assume_aligned(p, 16));
}
template <typename T>
__device__ __forceinline__ T* al16(T* p)
{
    return static_cast<T*>(__builtin_assume_aligned(p, 16));
}

// 128-bit LDS accesses to the object store: every 4-vector and spinor there
// starts on a 16-byte boundary, and the 16-bit immediate offset of a 128-bit
// access reaches every object of an event's store from one base address.
typedef double mf_d2 __attribute__((ext_vector_type(2), __may_alias__));
typedef float mf_f4 __attribute__((ext_vector_type(4), __may_alias__));

__device__ __forceinline__ void ld4(const double* p, double* o)
{
    const mf_d2 a = reinterpret_cast<const mf_d2*>(p)[0], b = reinterpret_cast<const mf_d2*>(p)[1];
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ __forceinline__ void ld4(const float* p, float* o)
{
    const mf_f4 a = *reinterpret_cast<const mf_f4*>(p);
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
}
__device__ __forceinline__ void st4(double* p, double a0, double a1, double a2, double a3)
{
    mf_d2 a, b;
    a.x = a0; a.y = a1; b.x = a2; b.y = a3;
    reinterpret_cast<mf_d2*>(p)[0] = a;
    reinterpret_cast<mf_d2*>(p)[1] = b;
}
__device__ __forceinline__ void st4(float* p, float a0, float a1, float a2, float a3)
{
    mf_f4 a;
    a.x = a0; a.y = a1; a.z = a2; a.w = a3;
    *reinterpret_cast<mf_f4*>(p) = a;
}
// complex 4-spinor, re/im interleaved
template <typename T>
__device__ __forceinline__ void ldspin(const T* p, cplx<T>* s)
{
    T a[4], b[4];
    ld4(p, a);
    ld4(p + 4, b);
    s[0] = cplx<T>(a[0], a[1]); s[1] = cplx<T>(a[2], a[3]);
    s[2] = cplx<T>(b[0], b[1]); s[3] = cplx<T>(b[2], b[3]);
}
template <typename T>
__device__ __forceinline__ void stspin(T* p, const cplx<T>* s)
{
    st4(p, s[0].x, s[0].y, s[1].x, s[1].y);
    st4(p + 4, s[2].x, s[2].y, s[3].x, s[3].y);
}

// The object store keeps each region chunk-major: of a region of N objects
// (4-vectors of 4 values, spinors of 8), 16-byte chunk c of object i lies at
// chunk c N + i of the region.  Lanes that read or write different objects of
// a region then touch consecutive 16-byte words, and up to 16 distinct
// objects per quarter wave fall in distinct LDS banks (a 32-byte FP64 4-vector
// per object would put objects 256 bytes apart in the same banks).  p points
// at chunk 0 of the object; the other chunks follow at a stride of N chunks,
// which the immediate offset of the access carries.
template <int N>
__device__ __forceinline__ void ld4s(const double* p, double* o)
{
    const mf_d2 a = reinterpret_cast<const mf_d2*>(p)[0], b = reinterpret_cast<const mf_d2*>(p + 2 * N)[0];
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
template <int N>
__device__ __forceinline__ void ld4s(const float* p, float* o)
{
    ld4(p, o);
}
template <int N>
__device__ __forceinline__ void st4s(double* p, double a0, double a1, double a2, double a3)
{
    mf_d2 a, b;
    a.x = a0; a.y = a1; b.x = a2; b.y = a3;
    reinterpret_cast<mf_d2*>(p)[0] = a;
    reinterpret_cast<mf_d2*>(p + 2 * N)[0] = b;
}
template <int N>
__device__ __forceinline__ void st4s(float* p, float a0, float a1, float a2, float a3)
{
    st4(p, a0, a1, a2, a3);
}
template <int N>
__device__ __forceinline__ void ldspins(const double* p, cplx<double>* s)
{
    for (int c = 0; c < 4; ++c) {
        const mf_d2 a = reinterpret_cast<const mf_d2*>(p + 2 * N * c)[0];
        s[c] = cplx<double>(a.x, a.y);
    }
}
template <int N>
__device__ __forceinline__ void ldspins(const float* p, cplx<float>* s)
{
    const mf_f4 a = *reinterpret_cast<const mf_f4*>(p), b = *reinterpret_cast<const mf_f4*>(p + 4 * N);
    s[0] = cplx<float>(a.x, a.y); s[1] = cplx<float>(a.z, a.w);
    s[2] = cplx<float>(b.x, b.y); s[3] = cplx<float>(b.z, b.w);
}
template <int N>
__device__ __forceinline__ void stspins(double* p, const cplx<double>* s)
{
    for (int c = 0; c < 4; ++c) {
        mf_d2 a;
        a.x = s[c].x; a.y = s[c].y;
        reinterpret_cast<mf_d2*>(p + 2 * N * c)[0] = a;
    }
}
template <int N>
__device__ __forceinline__ void stspins(float* p, const cplx<float>* s)
{
    mf_f4 a, b;
    a.x = s[0].x; a.y = s[0].y; a.z = s[1].x; a.w = s[1].y;
    b.x = s[2].x; b.y = s[2].y; b.z = s[3].x; b.w = s[3].y;
    *reinterpret_cast<mf_f4*>(p) = a;
    *reinterpret_cast<mf_f4*>(p + 4 * N) = b;
}

// Helicity pattern of the sub-sequence at positions start .. start+len-1 of a
// gluon sequence whose pattern is hm (bit k: the gluon at position k), in
// the order of the sub-sequence's stored orientation (rev: stored reversed).
__device__ __forceinline__ unsigned sub_pattern(unsigned hm, int start, int len, unsigned rev)
{
    const unsigned x = (hm >> start) & ((1u << len) - 1u);
    return rev ? (__brev(x) >> (32 - len)) : x;
}

// One complex amplitude (re, im) to device memory as a single store.
__device__ __forceinline__ void stj(double* p, double re, double im)
{
    mf_d2 v;
    v.x = re;
    v.y = im;
    *reinterpret_cast<mf_d2*>(p) = v;
}
typedef float mf_f2 __attribute__((ext_vector_type(2), __may_alias__));
__device__ __forceinline__ void stj(float* p, float re, float im)
{
    mf_f2 v;
    v.x = re;
    v.y = im;
    *reinterpret_cast<mf_f2*>(p) = v;
}

// (ar, ai) = c^mu j_mu for complex c and a real 4-vector j held in registers.
template <typename T>
__device__ __forceinline__ void cdot_set(const T* j, const cplx<T>* c, T& ar, T& ai)
{
    ar = c[0].x * j[0] - c[1].x * j[1] - c[2].x * j[2] - c[3].x * j[3];
    ai = c[0].y * j[0] - c[1].y * j[1] - c[2].y * j[2] - c[3].y * j[3];
}

// (ar, ai) += SGN c^mu j_mu as one multiply-add chain per component.
template <int SGN, typename T>
__device__ __forceinline__ void cdot_fma(const T* j, const cplx<T>* c, T& ar, T& ai)
{
    const T s = (T)SGN;
    ar += (s * c[0].x) * j[0];
    ar -= (s * c[1].x) * j[1];
    ar -= (s * c[2].x) * j[2];
    ar -= (s * c[3].x) * j[3];
    ai += (s * c[0].y) * j[0];
    ai -= (s * c[1].y) * j[1];
    ai -= (s * c[2].y) * j[2];
    ai -= (s * c[3].y) * j[3];
}

// W = gamma.e v = ((e.sigma) vR, (e.sigmabar) vL) for a real 4-vector e.
template <typename T>
__host__ __device__ __forceinline__ void slashcol(const T* e, const cplx<T>* v, cplx<T>* W)
{
    const T ep = e[0] + e[3], em = e[0] - e[3];
    // W0 = (e0 - e3) v2 + (-e1 + i e2) v3
    W[0] = cplx<T>(em * v[2].x - e[1] * v[3].x - e[2] * v[3].y, em * v[2].y - e[1] * v[3].y + e[2] * v[3].x);
    // W1 = (-e1 - i e2) v2 + (e0 + e3) v3
    W[1] = cplx<T>(-e[1] * v[2].x + e[2] * v[2].y + ep * v[3].x, -e[1] * v[2].y - e[2] * v[2].x + ep * v[3].y);
    // W2 = (e0 + e3) v0 + (e1 - i e2) v1
    W[2] = cplx<T>(ep * v[0].x + e[1] * v[1].x + e[2] * v[1].y, ep * v[0].y + e[1] * v[1].y - e[2] * v[1].x);
    // W3 = (e1 + i e2) v0 + (e0 - e3) v1
    W[3] = cplx<T>(e[1] * v[0].x - e[2] * v[0].y + em * v[1].x, e[1] * v[0].y + e[2] * v[0].x + em * v[1].y);
}

template <typename T>
__host__ __device__ __forceinline__ void rowdotcol(const cplx<T>* a, const cplx<T>* b, T& ar, T& ai)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ar += a[i].x * b[i].x - a[i].y * b[i].y;
        ai += a[i].x * b[i].y + a[i].y * b[i].x;
    }
}

// Real linear polarisations transverse to the 3-momentum of p (zero time
// component): h = 0 -> (0, cos th cos ph, cos th sin ph, -sin th),
// h = 1 -> (0, -sin ph, cos ph, 0).  Built in double from the momentum.
template <typename T>
__device__ __forceinline__ void linear_pol(const double* p, int h, T* e)
{
    const double pt2 = p[1] * p[1] + p[2] * p[2];
    const double pt = sqrt(pt2);
    const double kk = sqrt(pt2 + p[3] * p[3]);
    const bool has_pt = pt > 0.0;
    const double cph = has_pt ? p[1] / pt : 1.0;
    const double sph = has_pt ? p[2] / pt : 0.0;
    const double cth = p[3] / kk, sth = pt / kk;
    e[0] = (T)0;
    e[1] = (T)(h ? -sph : cth * cph);
    e[2] = (T)(h ? cph : cth * sph);
    e[3] = (T)(h ? 0.0 : -sth);
}

// Spinors with spin quantised along z in the rest frame, boosted:
//   u = (sqrt(p.sigma) xi, sqrt(p.sigmabar) xi),  v = (sqrt(p.sigma) xi, -sqrt(p.sigmabar) xi),
//   sqrt(p.sigma) = (p.sigma + m)/sqrt(2(E+m)),  xi_0 = (1, 0), xi_1 = (0, 1).
__host__ __device__ __forceinline__ void sqrt_blocks(const double* p, double m, int s, double* A, double* B)
{
    const double n = 1.0 / sqrt(2.0 * (p[0] + m));
    // columns s of (p.sigma + m) and (p.sigmabar + m), as (re, im) pairs
    if (s == 0) {
        A[0] = (p[0] - p[3] + m) * n; A[1] = 0.0;
        A[2] = -p[1] * n;             A[3] = -p[2] * n;
        B[0] = (p[0] + p[3] + m) * n; B[1] = 0.0;
        B[2] = p[1] * n;              B[3] = p[2] * n;
    } else {
        A[0] = -p[1] * n;             A[1] = p[2] * n;
        A[2] = (p[0] + p[3] + m) * n; A[3] = 0.0;
        B[0] = p[1] * n;              B[1] = -p[2] * n;
        B[2] = (p[0] - p[3] + m) * n; B[3] = 0.0;
    }
}

// ubar = u^dagger gamma^0 = (conj(uR), conj(uL)).
template <typename T>
__host__ __device__ __forceinline__ void spinor_ubar(const double* p, double m, int s, cplx<T>* ub)
{
    double A[4], B[4];
    sqrt_blocks(p, m, s, A, B);
    ub[0] = cplx<T>((T)B[0], (T)-B[1]);
    ub[1] = cplx<T>((T)B[2], (T)-B[3]);
    ub[2] = cplx<T>((T)A[0], (T)-A[1]);
    ub[3] = cplx<T>((T)A[2], (T)-A[3]);
}

template <typename T>
__host__ __device__ __forceinline__ void spinor_v(const double* p, double m, int s, cplx<T>* v)
{
    double A[4], B[4];
    sqrt_blocks(p, m, s, A, B);
    v[0] = cplx<T>((T)A[0], (T)A[1]);
    v[1] = cplx<T>((T)A[2], (T)A[3]);
    v[2] = cplx<T>((T)-B[0], (T)-B[1]);
    v[3] = cplx<T>((T)-B[2], (T)-B[3]);
}

// ---------------------------------------------------------------------------
// Philox4x32-10: 10 rounds of (c0..c3) -> (hi(M1 c2)^c1^k0, lo(M1 c2), hi(M0 c0)^c3^k1, lo(M0 c0)),
// M0 = 0xD2511F53, M1 = 0xCD9E8D57, key bumped by (0x9E3779B9, 0xBB67AE85).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t* r)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        // one 32 x 32 -> 64-bit multiply each (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    r[0] = c0; r[1] = c1; r[2] = c2; r[3] = c3;
}

// Monte Carlo over helicities: the configuration of event `event` (bit 0 top
// spin, bit 1 antitop spin, bit 2 + g gluon g's linear polarisation), uniform
// over n_hel: Philox block 0x80000002 of its counter, k the 53-bit integer of
// the first word pair, h = (k n_hel) >> 53 (Sec. 3.2 on Fig. 4 names the
// sampling of helicity configurations).
__device__ __forceinline__ int hel_config(uint64_t event, uint64_t seed, uint32_t iter, int n_hel)
{
    uint32_t r[4];
    philox4x32_10((uint32_t)event, (uint32_t)(event >> 32), iter, 0x80000002u, (uint32_t)seed,
                  (uint32_t)(seed >> 32), r);
    const uint64_t k = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
    return (int)((k * (uint64_t)n_hel) >> 53);
}

// ---------------------------------------------------------------------------
// Compensated accumulation.
// ---------------------------------------------------------------------------
struct Neumaier {
    double s, c;
};

__device__ __forceinline__ void nm_add(Neumaier& a, double v)
{
    const double t = a.s + v;
    if (fabs(a.s) >= fabs(v))
        a.c += (a.s - t) + v;
    else
        a.c += (v - t) + a.s;
    a.s = t;
}

// Merge two compensated partial sums (TwoSum of the leading parts).
__device__ __forceinline__ Neumaier nm_merge(Neumaier a, Neumaier b)
{
    const double s = a.s + b.s;
    const double bb = s - a.s;
    const double err = (a.s - (s - bb)) + (b.s - bb);
    Neumaier r;
    r.s = s;
    r.c = a.c + b.c + err;
    return r;
}

}  // namespace mf
