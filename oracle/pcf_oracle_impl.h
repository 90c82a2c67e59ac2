/*
 * pcf_oracle_impl.h -- key-type template of the oracle, included twice by
 * pcf_oracle.c (once for fp64 keys, once for uint64 keys).
 *
 * TEST INFRASTRUCTURE ONLY (see pcf_oracle.h).
 *
 * The includer defines:
 *   KEY     the key type (double or uint64_t)
 *   SUFFIX  a name suffix (f64 or u64)
 *   IS_F64  1 for fp64 keys, 0 for uint64 keys
 */

#define OR_CAT2(a, b) a##_##b
#define OR_CAT(a, b) OR_CAT2(a, b)
#define FN(name) OR_CAT(name, SUFFIX)
#define REC FN(rec)
#define VEC FN(vec)

/* A key travelling with its payload word. */
typedef struct {
    KEY k;
    uint32_t v;
} REC;

/* A growable bucket, c_j in Algorithm 1 (Sec. 3.2). */
typedef struct {
    REC *p;
    uint64_t len, cap;
} VEC;

static int FN(vec_push)(VEC *c, REC r)
{
    if (c->len == c->cap) {
        uint64_t cap = c->cap ? 2 * c->cap : 4;
        REC *p = (REC *)realloc(c->p, cap * sizeof(REC));
        if (!p)
            return PCFO_ERR_NOMEM;
        c->p = p;
        c->cap = cap;
    }
    c->p[c->len++] = r;
    return PCFO_OK;
}

/* Keys must be finite and not -0.0 so that the ascending order is unique. */
static int FN(key_valid)(KEY k)
{
#if IS_F64
    uint64_t bits;
    memcpy(&bits, &k, sizeof bits);
    if (!isfinite(k))
        return 0;
    if (bits == 0x8000000000000000ULL)
        return 0;
    return 1;
#else
    (void)k;
    return 1;
#endif
}

/*
 * Standard sort (Sec. 3.1 allows any sort with guarantees): a textbook
 * top-down merge sort, stable, O(n log n) in the worst case.  Sorts a[0..n)
 * by key; equal keys keep their order.  tmp must hold n records.
 */
static void FN(merge_sort)(REC *a, REC *tmp, uint64_t n)
{
    if (n < 2)
        return;
    uint64_t h = n / 2;
    FN(merge_sort)(a, tmp, h);
    FN(merge_sort)(a + h, tmp, n - h);
    uint64_t i = 0, j = h, o = 0;
    while (i < h && j < n) {
#ifdef PCFO_PLANT_UNSTABLE
        if (a[j].k <= a[i].k) /* planted mistake: ties taken from the right half */
#else
        if (a[j].k < a[i].k)
#endif
            tmp[o++] = a[j++];
        else
            tmp[o++] = a[i++];
    }
    while (i < h)
        tmp[o++] = a[i++];
    while (j < n)
        tmp[o++] = a[j++];
    memcpy(a, tmp, n * sizeof(REC));
}

/*
 * The bin function i(x) of Sec. 3.3, 0-based:
 *   bin(v) = min(beta, floor(RN(off(v) * s))),  s = RN(beta / RN(x_max - x_min)),
 * with off(v) = RN(v - x_min).  When x_max - x_min overflows (fp64 only), both
 * terms are halved first: off(v) = RN(v/2 - x_min/2), s = RN(beta / RN(x_max/2 -
 * x_min/2)).  For uint64 keys off(v) is the exact integer difference rounded to
 * fp64.  Returns 0 when s is not finite (the node is then a bucketing failure).
 */
typedef struct {
    KEY lo;
    double s;
    int halves;
    uint64_t beta;
} FN(binfn);

static int FN(bin_setup)(FN(binfn) *f, KEY mn, KEY mx, uint64_t beta)
{
    double d;
    f->lo = mn;
    f->beta = beta;
    f->halves = 0;
#if IS_F64
    d = mx - mn;
    if (isinf(d)) {
        f->halves = 1;
        d = mx * 0.5 - mn * 0.5;
    }
#else
    d = (double)(mx - mn);
#endif
#ifdef PCFO_PLANT_SCALE_OPERAND
    f->s = (double)(beta / 2 + 1) / d; /* planted mistake: wrong numerator */
#else
    f->s = (double)beta / d;
#endif
    return isfinite(f->s) ? 1 : 0;
}

/* Position of v in bin units: RN(RN(v - x_min) * s), before the floor. */
static double FN(pos)(const FN(binfn) *f, KEY v)
{
    double off;
#if IS_F64
    if (f->halves)
#ifdef PCFO_PLANT_HALF_OFFSET
        off = v * 0.5 - f->lo; /* planted mistake: only the key is halved */
#else
        off = v * 0.5 - f->lo * 0.5;
#endif
    else
        off = v - f->lo;
#else
    off = (double)(v - f->lo);
#endif
    return off * f->s;
}

static uint64_t FN(bin)(const FN(binfn) *f, KEY v)
{
    double p = FN(pos)(f, v);
    uint64_t k = (uint64_t)floor(p);
#ifdef PCFO_PLANT_BIN_PLUS_ONE
    k += 1; /* planted mistake: the paper's 1-based bin leaks into 0-based code */
#endif
    return k < f->beta ? k : f->beta;
}

/*
 * Spline inference (App. A.5), 0-based: the key's bin k = min(beta, floor(p)),
 * its relative position inside the bin frac = p - k (exact in fp64), and
 * F(x) alpha = b_{k-1} + frac * (b_k - b_{k-1}) with b_{-1} = 0; the bucket is
 * floor(F(x) gamma).  Each step is one IEEE round-to-nearest operation, in
 * this order: t = frac * c, v = b_{k-1} + t, u = v * gamma, w = u / alpha.
 * Every step is monotone and v never exceeds b_k, so buckets are
 * non-decreasing in the key and agree with the PCF's at the bin thresholds.
 */
static uint64_t FN(spline_bucket)(const FN(binfn) *f, const uint64_t *b, uint64_t alpha,
                                  uint64_t gamma, KEY v)
{
    double p = FN(pos)(f, v);
    uint64_t k = (uint64_t)floor(p);
    if (k > f->beta)
        k = f->beta;
    double frac = p - (double)k;
#ifdef PCFO_PLANT_SPLINE_UPPER
    uint64_t lo = b[k]; /* planted mistake: interpolate from the bin's upper value */
#else
    uint64_t lo = k ? b[k - 1] : 0;
#endif
    uint64_t c = b[k] - (k ? b[k - 1] : 0);
#ifdef PCFO_PLANT_SPLINE_NOFRAC
    double t = 0.0; /* planted mistake: the interpolation term is dropped */
#else
    double t = frac * (double)c;
#endif
    double vv = (double)lo + t;
    double u = vv * (double)gamma;
    double w = u / (double)alpha;
    uint64_t q = (uint64_t)floor(w);
    return q < gamma ? q : gamma;
}

/* Quantization condition of App. A.4 for the node interval [lo, hi]. */
static double FN(quant_lhs)(uint64_t beta, KEY lo, KEY hi)
{
#if IS_F64
    return pcfo_quant_lhs_f64(beta, lo, hi);
#else
    /* integer keys: every quantization cell has width 1 */
    return (double)beta / (double)(hi - lo);
#endif
}

typedef struct {
    KEY mn, mx;
    double s;
    int halves;
} FN(lvl_scalars);

#define ST_BUCKETED 0
#define ST_SINGLE 1
#define ST_NONFINITE 2

/*
 * One model-based bucketing (Algorithm 1, CDF-Model + Append loop; PCF
 * training and inference of Sec. 3.3) of a[0..n) in place: on return a[] holds
 * the buckets c_0 .. c_gamma concatenated, each in input order, and sizes[j] =
 * |c_j|.  b_out / T_out / sample_pos_out are optional trace arrays.
 */
static int FN(bucketize)(REC *a, uint64_t n, uint64_t node_seed, uint64_t alpha, uint64_t beta,
                         uint64_t gamma, const uint64_t *sample_idx, uint64_t *b_out,
                         uint64_t *T_out, uint64_t *sizes, uint64_t *sample_pos_out,
                         FN(lvl_scalars) *sc, int *status, int model)
{
    uint64_t i, j;
    /* x_min and x_max of the whole current array (Sec. 3.3). */
    KEY mn = a[0].k, mx = a[0].k;
    for (i = 1; i < n; i++) {
        if (a[i].k < mn)
            mn = a[i].k;
        if (a[i].k > mx)
            mx = a[i].k;
    }
    sc->mn = mn;
    sc->mx = mx;
    sc->s = 0.0;
    sc->halves = 0;
    if (mn == mx) {
        *status = ST_SINGLE;
        return PCFO_OK;
    }
    FN(binfn) f;
    int ok = FN(bin_setup)(&f, mn, mx, beta);
    sc->s = f.s;
    sc->halves = f.halves;
    if (!ok) {
        *status = ST_NONFINITE;
        return PCFO_OK;
    }

    /* Training by counting: b_i = #{ j : i(a_j) <= i } over alpha samples. */
    uint64_t *b = b_out ? b_out : (uint64_t *)malloc((beta + 1) * sizeof(uint64_t));
    uint64_t *T = T_out ? T_out : (uint64_t *)malloc((beta + 1) * sizeof(uint64_t));
    if (!b || !T) {
        if (!b_out)
            free(b);
        if (!T_out)
            free(T);
        return PCFO_ERR_NOMEM;
    }
    memset(b, 0, (beta + 1) * sizeof(uint64_t));
    for (j = 0; j < alpha; j++) {
        uint64_t pos = sample_idx ? sample_idx[j] : pcfo_sample_index(node_seed, j, n);
        if (sample_pos_out)
            sample_pos_out[j] = pos;
        b[FN(bin)(&f, a[pos].k)] += 1;
    }
#ifdef PCFO_PLANT_EXCLUSIVE_PREFIX
    /* planted mistake: exclusive instead of inclusive prefix */
    {
        uint64_t run = 0;
        for (i = 0; i <= beta; i++) {
            uint64_t h = b[i];
            b[i] = run;
            run += h;
        }
    }
#else
    for (i = 1; i <= beta; i++)
        b[i] += b[i - 1];
#endif

    /* Inference: bucket index floor(F(x) gamma) = floor(b_{i(x)} gamma / alpha). */
    for (i = 0; i <= beta; i++)
#ifdef PCFO_PLANT_T_CEIL
        T[i] = (uint64_t)(((unsigned __int128)b[i] * gamma + alpha - 1) / alpha); /* planted */
#else
        T[i] = (uint64_t)(((unsigned __int128)b[i] * gamma) / alpha);
#endif

    /* Append every key, in input order, to its bucket. */
    VEC *c = (VEC *)calloc(gamma + 1, sizeof(VEC));
    int rc = c ? PCFO_OK : PCFO_ERR_NOMEM;
    for (i = 0; i < n && rc == PCFO_OK; i++) {
        uint64_t q = model == PCFO_MODEL_SPLINE ? FN(spline_bucket)(&f, b, alpha, gamma, a[i].k)
                                                : T[FN(bin)(&f, a[i].k)];
        rc = FN(vec_push)(&c[q], a[i]);
    }

    /* Concatenate the buckets back into a[]. */
    if (rc == PCFO_OK) {
        uint64_t pos = 0;
        for (j = 0; j <= gamma; j++) {
            if (c[j].len)
                memcpy(a + pos, c[j].p, c[j].len * sizeof(REC));
            sizes[j] = c[j].len;
            pos += c[j].len;
        }
    }
    if (c) {
        for (j = 0; j <= gamma; j++)
            free(c[j].p);
        free(c);
    }
    if (!b_out)
        free(b);
    if (!T_out)
        free(T);
    *status = ST_BUCKETED;
    return rc;
}

typedef struct {
    uint64_t seed, segment, tau;
    int model;
} FN(ctx);

/*
 * Learned-Sort (Algorithm 1) with the parameter rule of the PCF theorems:
 * alpha = beta = gamma = delta = floor(n^{3/4}).  Sorts a[0..n) in place.
 * `off` is the position of a[0] in the whole output, used to name the node.
 */
static int FN(ls)(REC *a, REC *tmp, uint64_t n, const FN(ctx) *cx, uint64_t depth, uint64_t off,
                  pcfo_stats *st)
{
    if (depth > st->max_depth)
        st->max_depth = depth;
    if (n < cx->tau) {
        FN(merge_sort)(a, tmp, n);
        st->small_sorts++;
        return PCFO_OK;
    }
    uint64_t r = pcfo_root34(n);
    uint64_t alpha = r, beta = r, gamma = r, delta = r;
    uint64_t *sizes = (uint64_t *)malloc((gamma + 1) * sizeof(uint64_t));
    if (!sizes)
        return PCFO_ERR_NOMEM;
    FN(lvl_scalars) sc;
    int status;
    int rc = FN(bucketize)(a, n, pcfo_node_seed(cx->seed, cx->segment, depth, off), alpha, beta,
                           gamma, NULL, NULL, NULL, sizes, NULL, &sc, &status, cx->model);
    if (rc != PCFO_OK) {
        free(sizes);
        return rc;
    }
    if (status == ST_SINGLE) {
        st->single_valued++;
        free(sizes);
        return PCFO_OK;
    }
    if (status == ST_NONFINITE) {
        st->nonfinite_scale++;
        FN(merge_sort)(a, tmp, n);
        free(sizes);
        return PCFO_OK;
    }
    st->levels++;
    double q = FN(quant_lhs)(beta, sc.mn, sc.mx);
    if (q > st->max_quant_lhs)
        st->max_quant_lhs = q;

    /* Sort every bucket (standard sort if |c_j| >= delta, else recurse);
       the buckets are already concatenated in place. */
    uint64_t pos = 0;
    for (uint64_t j = 0; j <= gamma && rc == PCFO_OK; j++) {
        uint64_t m = sizes[j];
#ifdef PCFO_PLANT_NO_FALLBACK
        if (0) { /* planted mistake: failed buckets recurse instead of the standard sort */
#else
        if (m >= delta) {
#endif
            FN(merge_sort)(a + pos, tmp, m);
            st->fail_sorts++;
            st->fail_keys += m;
        } else if (m > 0) {
            rc = FN(ls)(a + pos, tmp, m, cx, depth + 1, off + pos, st);
        }
        pos += m;
    }
    free(sizes);
    return rc;
}

static int FN(load)(const KEY *keys, const uint32_t *vals, uint64_t n, REC **out)
{
    REC *a = (REC *)malloc((n ? n : 1) * sizeof(REC));
    if (!a)
        return PCFO_ERR_NOMEM;
    for (uint64_t i = 0; i < n; i++) {
        if (!FN(key_valid)(keys[i])) {
            free(a);
            return PCFO_ERR_INVALID_KEY;
        }
        a[i].k = keys[i];
        a[i].v = vals ? vals[i] : 0u;
    }
    *out = a;
    return PCFO_OK;
}

static void FN(store)(const REC *a, uint64_t n, KEY *keys, uint32_t *vals)
{
    for (uint64_t i = 0; i < n; i++) {
        keys[i] = a[i].k;
        if (vals)
            vals[i] = a[i].v;
    }
}

static int FN(sort_entry)(const KEY *keys_in, const uint32_t *vals_in, KEY *keys_out,
                          uint32_t *vals_out, uint64_t n, uint64_t seed, uint64_t segment,
                          uint64_t tau, int model, pcfo_stats *st)
{
    REC *a = NULL;
    int rc = FN(load)(keys_in, vals_in, n, &a);
    if (rc != PCFO_OK)
        return rc;
    REC *tmp = (REC *)malloc((n ? n : 1) * sizeof(REC));
    if (!tmp) {
        free(a);
        return PCFO_ERR_NOMEM;
    }
    FN(ctx) cx = {seed, segment, tau, model};
    rc = FN(ls)(a, tmp, n, &cx, 0, 0, st);
    if (rc == PCFO_OK)
        FN(store)(a, n, keys_out, vals_out);
    free(tmp);
    free(a);
    return rc;
}

static int FN(level_entry)(const KEY *keys, const uint32_t *vals, uint64_t n, uint64_t node_seed,
                           pcfo_level_io *io)
{
    REC *a = NULL;
    int rc = FN(load)(keys, vals, n, &a);
    if (rc != PCFO_OK)
        return rc;
    FN(lvl_scalars) sc;
    int status;
    rc = FN(bucketize)(a, n, node_seed, io->alpha, io->beta, io->gamma, io->sample_idx, io->b,
                       io->T, io->sizes, io->sample_pos, &sc, &status, io->model);
    if (rc == PCFO_OK) {
        memcpy(&io->min_bits, &sc.mn, sizeof(uint64_t));
        memcpy(&io->max_bits, &sc.mx, sizeof(uint64_t));
        io->scale = sc.s;
        io->halves = sc.halves;
        io->status = status;
        /* bucketed: the concatenated buckets; otherwise the input unchanged */
        FN(store)(a, n, (KEY *)io->part_keys, io->part_vals);
    }
    free(a);
    return rc;
}

#undef ST_BUCKETED
#undef ST_SINGLE
#undef ST_NONFINITE
#undef VEC
#undef REC
#undef FN
#undef OR_CAT
#undef OR_CAT2
