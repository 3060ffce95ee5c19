// Host replay of the kernels' loop nests over the device arrays, with every index
// computed by the functions the kernels use (hefk_layout.hpp) and checked against
// the size the host code allocates.  Built with AddressSanitizer and UBSan.
//
// stdin, one configuration per line:
//   n resident n_steps sample_every ckpt_every rows_in_lds
// (resident: blocks resident at once, as the occupancy query would give; ckpt_every 0:
// no checkpoints).  stdout: one line per configuration, "ok grid=G", or a message and
// exit status 1 at the first violation.
//
// Replayed: init_kernel (one walker per thread), propagate_kernel (persistent blocks
// over chunks, tail lanes shadowing the last walker, the sampling and checkpoint
// counters of the step loop, partial rows in LDS or in the workspace), merge_kernel,
// and the gradient's two reverse sweeps (segment tape, stored trajectory).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hefk_layout.hpp"

using namespace hefk;

static void fail(const char* what, long long idx, long long size)
{
    std::printf("index %lld outside [0, %lld) in %s\n", idx, size, what);
    std::exit(1);
}

// counts the accesses to each element of one array
struct Arr {
    const char* name;
    std::vector<unsigned> hits;
    Arr(const char* nm, size_t size) : name(nm), hits(size, 0u) {}
    void at(long long idx)
    {
        if (idx < 0 || idx >= (long long)hits.size()) fail(name, idx, (long long)hits.size());
        ++hits[(size_t)idx];
    }
    void expect_each(unsigned times, const char* what) const
    {
        for (size_t k = 0; k < hits.size(); ++k)
            if (hits[k] != times) {
                std::printf("%s: element %zu of %s hit %u times, expected %u\n", what, k, name, hits[k], times);
                std::exit(1);
            }
    }
};

static void run(long long n, long long resident, int n_steps, int se, int ce, bool rows_in_lds)
{
    const int64_t n_chunks = layout::chunks(n);
    const int64_t ns = n_steps / se + 1;
    const int64_t n_ckpt = ce ? n_steps / ce + 1 : 0;

    // init_kernel: grid = chunks(n), one walker per thread
    {
        Arr x("x", 6 * (size_t)n), el("el", (size_t)n), lnw("lnw", (size_t)n);
        for (int64_t b = 0; b < n_chunks; ++b)
            for (uint32_t t = 0; t < (uint32_t)layout::kLanes; ++t) {
                const int64_t i = layout::walker(b, t);
                if (i >= n) continue;
                for (int k = 0; k < 6; ++k) x.at(layout::coord(k, n, i));
                el.at(i);
                lnw.at(i);
            }
        x.expect_each(1, "init writes");
        el.expect_each(1, "init writes");
        lnw.expect_each(1, "init writes");
    }

    // propagate_kernel
    const int64_t G = layout::grid(n_chunks, resident);
    if (G < 1 || G > n_chunks || G > resident) {
        std::printf("grid %lld for %lld chunks and %lld resident blocks\n", (long long)G, (long long)n_chunks,
                    resident);
        std::exit(1);
    }
    // the step loop's counters are the same for every chunk: the sample rows and
    // checkpoint rows it reaches, in order
    std::vector<int> rows_hit, ckpt_hit;
    {
        int row = 1, until_sample = se, until_ckpt = ce, crow = 1;
        for (int k = 0; k < n_steps; ++k) {
            if (--until_sample == 0) {
                until_sample = se;
                rows_hit.push_back(row);
                ++row;
            }
            if (ce && --until_ckpt == 0) {
                until_ckpt = ce;
                ckpt_hit.push_back(crow);
                ++crow;
            }
        }
        if (row != ns || (ce && crow != n_ckpt)) {
            std::printf("step loop reached row %d of %lld, checkpoint %d of %lld\n", row, (long long)ns, crow,
                        (long long)n_ckpt);
            std::exit(1);
        }
    }
    Arr xr("x (read)", 6 * (size_t)n), lnwr("lnw (read)", (size_t)n);
    Arr xw("x (write)", 6 * (size_t)n), lnww("lnw (write)", (size_t)n), elw("el (write)", (size_t)n);
    // HEFK_LAYOUT_SHORT=1: the checkpoint array one element short (the replay must then fail)
    const char* short_env = std::getenv("HEFK_LAYOUT_SHORT");
    const size_t shortfall = (short_env && short_env[0] == '1' && ce) ? 1 : 0;
    Arr ck("ckpt", (size_t)n_ckpt * 7 * (size_t)n - shortfall);
    Arr parts("partials", layout::block_rows(G, ns));
    std::vector<unsigned> chunk_seen((size_t)n_chunks, 0u);
    for (int64_t b = 0; b < G; ++b) {
        const size_t rows_out = layout::block_rows(b, ns);
        Arr lds("rows in LDS", layout::row_offset(ns));
        std::vector<unsigned> row_written((size_t)ns, 0u);
        auto sample = [&](int row) {
            for (int e = 0; e < 8; ++e) {
                if (rows_in_lds)
                    lds.at((long long)(layout::row_offset(row) + e));
                else
                    parts.at((long long)(rows_out + layout::row_offset(row) + e));
            }
            ++row_written[(size_t)row];
        };
        for (int64_t c = b; c < n_chunks; c += G) {
            ++chunk_seen[(size_t)c];
            for (uint32_t t = 0; t < (uint32_t)layout::kLanes; ++t) {
                const int64_t i = layout::walker(c, t);
                const bool valid = i < n;
                const int64_t ii = valid ? i : n - 1;
                for (int k = 0; k < 6; ++k) xr.at(layout::coord(k, n, ii));
                lnwr.at(ii);
                if (ce && valid)
                    for (int k = 0; k < 7; ++k) ck.at(layout::coord(k, n, i));  // checkpoint row 0
                if (ce && valid)
                    for (int crow : ckpt_hit)
                        for (int k = 0; k < 7; ++k) ck.at((long long)(layout::ckpt_row(crow, n) + layout::coord(k, n, i)));
                if (valid) {
                    for (int k = 0; k < 6; ++k) xw.at(layout::coord(k, n, i));
                    lnww.at(i);
                    elw.at(i);
                }
            }
            sample(0);  // thread 0, once per chunk
            for (int row : rows_hit) sample(row);
        }
        for (int64_t r = 0; r < ns; ++r)
            if (row_written[(size_t)r] == 0) {
                std::printf("block %lld never wrote its sample row %lld\n", (long long)b, (long long)r);
                std::exit(1);
            }
        if (rows_in_lds) {
            lds.expect_each((unsigned)((n_chunks - b + G - 1) / G), "LDS rows");
            for (int64_t k = 0; k < ns * 8; ++k) parts.at((long long)(rows_out + k));  // the copy at the end
        }
    }
    for (int64_t c = 0; c < n_chunks; ++c)
        if (chunk_seen[(size_t)c] != 1) {
            std::printf("chunk %lld visited %u times\n", (long long)c, chunk_seen[(size_t)c]);
            std::exit(1);
        }
    xw.expect_each(1, "propagate writes");
    lnww.expect_each(1, "propagate writes");
    elw.expect_each(1, "propagate writes");
    if (ce) ck.expect_each(1, "checkpoint writes");
    if (rows_in_lds) parts.expect_each(1, "partial rows");

    // merge_kernel: one block per sample row, reading that row of every partial block
    {
        Arr pr("partials (merge)", layout::block_rows(G, ns));
        for (int64_t s = 0; s < ns; ++s)
            for (int64_t b = 0; b < G; ++b)
                for (int e = 0; e < 8; ++e) pr.at((long long)(layout::block_rows(b, ns) + layout::row_offset(s) + e));
        pr.expect_each(1, "merge reads");
    }

    // gradient sweeps (one thread per walker, grid chunks(n))
    if (ce) {
        const int64_t nt = ce == 1 ? 0 : (int64_t)(ce + 1) * 7 * n;  // the recomputing sweep's tape
        Arr ckr("ckpt (gradient)", (size_t)n_ckpt * 7 * (size_t)n), tape("tape", (size_t)nt);
        for (int64_t b = 0; b < n_chunks; ++b)
            for (uint32_t t = 0; t < (uint32_t)layout::kLanes; ++t) {
                const int64_t i = layout::walker(b, t);
                if (i >= n) continue;
                if (ce == 1) {
                    for (int j = n_steps; j >= 0; --j) {
                        for (int k = 0; k < 6; ++k) ckr.at((long long)(layout::ckpt_row(j, n) + layout::coord(k, n, i)));
                        if (j % se == 0) ckr.at((long long)(layout::ckpt_row(j, n) + layout::coord(6, n, i)));
                    }
                } else {
                    for (int seg = n_steps / ce - 1; seg >= 0; --seg) {
                        for (int k = 0; k < 7; ++k) ckr.at((long long)(layout::ckpt_row(seg, n) + layout::coord(k, n, i)));
                        for (int slot = 0; slot <= ce; ++slot)
                            for (int k = 0; k < 7; ++k)
                                tape.at((long long)(layout::ckpt_row(slot, n) + layout::coord(k, n, i)));
                    }
                }
                // the start-law score term reads checkpoint row 0
                for (int k = 0; k < 6; ++k) ckr.at((long long)(layout::ckpt_row(0, n) + layout::coord(k, n, i)));
            }
    }
    std::printf("ok grid=%lld\n", (long long)G);
}

int main()
{
    long long n, resident;
    int n_steps, se, ce, lds;
    while (std::scanf("%lld %lld %d %d %d %d", &n, &resident, &n_steps, &se, &ce, &lds) == 6) {
        run(n, resident, n_steps, se, ce, lds != 0);
        std::fflush(stdout);
    }
    return 0;
}
