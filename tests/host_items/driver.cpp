// Host build of the flash's per-mixture work items (flash_stages.hpp,
// srk_device.hpp), for checks that need a CPU: the item code run one mixture
// per thread under the address and undefined-behaviour sanitizers.  The
// stages run as in the plain form: every item of a stage steps to completion
// (the outbox entries of each step appended to the stage lists), then the
// next stage reads its lists.  Compiled once per component count (HOST_NC).
//
// Input file (little-endian): int64 n, int32 nc, int32 per_mixture, then the
// options as 8 int32 (max_pre_ss, max_ss, max_tr_sa, max_tr_split,
// max_polish, dem_every, keep_factor, unused) and 6 float64 (tol_sa_ss,
// tol_sa_tr, tol_split_ss, tol_split_tr, tol_polish, eps_tm), then z (n*nc),
// T (n), P (n), Tc, Pc, omega (nc or n*nc), kij (nc*nc or n*nc*nc).
// Output file: label (int8 n), beta (n), x (n*nc), y (n*nc), iters (int16
// n*8), status (uint16 n), flops (uint32 n), tm (n).
//   usage: driver_ncNC <in> <out> <threads> [nofill]
// The per-mixture records are filled with 0xff bytes first (so that a read
// before the write sees NaN and huge counters, not zeros), unless "nofill"
// is given (for the uninitialised-read sanitizer, which must see them
// unwritten).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "flash_stages.hpp"

using namespace ptf;

#ifndef HOST_NC
#error "HOST_NC must be defined"
#endif
constexpr int NC = HOST_NC;

template <typename T>
static void read_n(FILE *f, std::vector<T> &v, size_t n)
{
    v.resize(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
}

template <typename T>
static void write_v(FILE *f, const std::vector<T> &v)
{
    if (!v.empty()) fwrite(v.data(), sizeof(T), v.size(), f);
}

using HostLists = std::vector<std::vector<uint32_t>>;

static void collect(std::vector<std::pair<int, uint32_t>> &out, const Outbox &ob)
{
    if (ob.l0 >= 0) {
        out.push_back({ob.l0, ob.i0});
        if (ob.n0 == 2) out.push_back({ob.l0, ob.i0 + 1u});
    }
    if (ob.l1 >= 0) out.push_back({ob.l1, ob.i1});
}

template <class Item>
static void run_stage(const Ctx<NC> &c, HostLists &lists, int nthreads)
{
    std::vector<uint32_t> in;
    if (Item::LIST < 0) {
        in.resize((size_t)c.a.n);
        for (size_t k = 0; k < in.size(); ++k) in[k] = (uint32_t)k;
    } else {
        in = lists[Item::LIST < 0 ? 0 : Item::LIST];
        if (Item::LIST2 >= 0) {
            const auto &l2 = lists[Item::LIST2 < 0 ? 0 : Item::LIST2];
            in.insert(in.end(), l2.begin(), l2.end());
        }
    }
    std::vector<std::vector<std::pair<int, uint32_t>>> outs(nthreads);
    auto work = [&](int t) {
        for (size_t k = (size_t)t; k < in.size(); k += (size_t)nthreads) {
            Item it;
            it.ob.clear();
            if (!it.begin(c, in[k])) continue;
            for (int s = 0;; ++s) {
                it.ob.clear();
                const bool done = it.step(c);
                collect(outs[t], it.ob);
                if (done) break;
                if (s > 4 * kStepGuard) {
                    fprintf(stderr, "item %u of stage %d does not finish\n", in[k], Item::LIST);
                    abort();
                }
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nthreads; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
    for (auto &o : outs)
        for (auto &e : o) lists[e.first].push_back(e.second);
}

static bool fill_records(int argc, char **argv)
{
    return !(argc > 4 && std::strcmp(argv[4], "nofill") == 0);
}

int main(int argc, char **argv)
{
    if (argc < 4) {
        fprintf(stderr, "usage: %s <in> <out> <threads>\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n = 0;
    int32_t nc = 0, pm = 0, oi[8];
    double od[6];
    if (fread(&n, 8, 1, f) != 1 || fread(&nc, 4, 1, f) != 1 || fread(&pm, 4, 1, f) != 1 ||
        fread(oi, 4, 8, f) != 8 || fread(od, 8, 6, f) != 6)
        return 2;
    if (nc != NC || n < 0) {
        fprintf(stderr, "nc %d does not match this build (%d)\n", nc, NC);
        return 2;
    }
    const size_t un = (size_t)n, pn = pm ? un : 1;
    std::vector<double> z, T, P, Tc, Pc, om, K;
    read_n(f, z, un * NC);
    read_n(f, T, un);
    read_n(f, P, un);
    read_n(f, Tc, pn * NC);
    read_n(f, Pc, pn * NC);
    read_n(f, om, pn * NC);
    read_n(f, K, pn * NC * NC);
    fclose(f);

    std::vector<int8_t> label(un);
    std::vector<double> beta(un), x(un * NC), y(un * NC), tm(un);
    std::vector<int16_t> iters(un * 8);
    std::vector<uint16_t> status(un);
    std::vector<uint32_t> flops(un);
    std::vector<MixRec<NC>> rec(fill_records(argc, argv) ? un : 0);
    const bool fill = fill_records(argc, argv);
    MixRec<NC> *recp = fill ? rec.data() : (MixRec<NC> *)std::malloc(un * sizeof(MixRec<NC>) + 1);
    if (fill) std::memset((void *)recp, 0xff, un * sizeof(MixRec<NC>));

    Ctx<NC> c;
    std::memset((void *)&c, 0, sizeof(c));
    FlashArgs &a = c.a;
    a.n = n;
    a.z = z.data();
    a.T = T.data();
    a.P = P.data();
    a.max_pre_ss = oi[0];
    a.max_ss = oi[1];
    a.max_tr_sa = oi[2];
    a.max_tr_split = oi[3];
    a.max_polish = oi[4];
    a.dem_every = oi[5];
    a.keep_factor = 0;
    a.tol_sa_ss = od[0];
    a.tol_sa_tr = od[1];
    a.tol_split_ss = od[2];
    a.tol_split_tr = od[3];
    a.tol_polish = od[4];
    a.eps_tm = od[5];
    a.label = label.data();
    a.beta = beta.data();
    a.x = x.data();
    a.y = y.data();
    a.iters = iters.data();
    a.status = status.data();
    a.flops = flops.data();
    a.factor = nullptr;
    a.tm = tm.data();
    a.stability_only = 0;
    a.lnk0 = nullptr;
    a.hint = nullptr;
    c.pr = Props{Tc.data(), Pc.data(), om.data(), K.data()};
    c.rec = recp;

    const int nthreads = std::max(1, atoi(argv[3]));
    HostLists lists(L_COUNT);
    if (pm) {
        run_stage<FeedItem<NC, true>>(c, lists, nthreads);
        run_stage<PreSsItem<NC, true>>(c, lists, nthreads);
        run_stage<SaSsItem<NC, true>>(c, lists, nthreads);
        run_stage<SaTrItem<NC, true>>(c, lists, nthreads);
        run_stage<SaFinItem<NC, true>>(c, lists, nthreads);
        run_stage<SpSsItem<NC, true>>(c, lists, nthreads);
        run_stage<SpNtItem<NC, true>>(c, lists, nthreads);
    } else {
        run_stage<FeedItem<NC, false>>(c, lists, nthreads);
        run_stage<PreSsItem<NC, false>>(c, lists, nthreads);
        run_stage<SaSsItem<NC, false>>(c, lists, nthreads);
        run_stage<SaTrItem<NC, false>>(c, lists, nthreads);
        run_stage<SaFinItem<NC, false>>(c, lists, nthreads);
        run_stage<SpSsItem<NC, false>>(c, lists, nthreads);
        run_stage<SpNtItem<NC, false>>(c, lists, nthreads);
    }

    FILE *g = fopen(argv[2], "wb");
    if (!g) return 2;
    write_v(g, label);
    write_v(g, beta);
    write_v(g, x);
    write_v(g, y);
    write_v(g, iters);
    write_v(g, status);
    write_v(g, flops);
    write_v(g, tm);
    fclose(g);
    if (!fill) std::free(recp);
    return 0;
}
