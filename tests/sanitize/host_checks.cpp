// host_checks.cpp -- drives the library's host-only decision code (argument
// validation, operand overlap, default tile rules, the split-K plan, the
// edge split, the thin-product plan, the grouped list schedule and batch
// aliasing) from commands on stdin, one
// result line per command.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py, which checks
// the results against the library itself and against brute force.
//
//   V ta tb M N K alpha A lda B ldb beta C ldc -> validate status
//   O ta tb M N K alpha A lda B ldb C ldc      -> 1 if C overlaps A or B
//   D prec ta tb M N K                         -> built-in configuration
//   S M N K cus                                -> small_tile splits kc
//   E ta tb M N K                              -> 1 Mm Nm (edge split) or 0
//   T ta tb M N K lda ldb ldc cus              -> ok rows splits kc bytes gather (thin)
//   L G n cost_1 .. cost_n                     -> work-group of each item
//   B nc na (lo hi owner) x (nc + na)          -> culprit kind
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "host_common.hpp"
#include "rules.hpp"

using namespace mgemm;

static const float* fp(unsigned long long v) { return reinterpret_cast<const float*>(v); }

int main() {
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        char op = 0;
        in >> op;
        if (op == 'V' || op == 'O') {
            char ta, tb;
            long long M, N, K, lda, ldb, ldc;
            float alpha, beta = 0.0f;
            unsigned long long A, B, C;
            in >> ta >> tb >> M >> N >> K >> alpha >> A >> lda >> B >> ldb;
            if (op == 'V') in >> beta;
            in >> C >> ldc;
            if (!in) { std::printf("bad\n"); continue; }
            if (op == 'V') {
                std::string why;
                std::printf("%d\n", validate(ta, tb, M, N, K, alpha, fp(A), lda, fp(B), ldb, beta,
                                             fp(C), ldc, why));
            } else {
                std::printf("%d\n", overlaps(trans_code(ta), trans_code(tb), M, N, K, alpha,
                                             fp(A), lda, fp(B), ldb, fp(C), ldc) ? 1 : 0);
            }
        } else if (op == 'D') {
            int prec;
            char ta, tb;
            long long M, N, K;
            in >> prec >> ta >> tb >> M >> N >> K;
            const bool a = trans_code(ta) == 1, b = trans_code(tb) == 1;
            const int c = prec == 0   ? f32_default_config(a, b, M, N, K)
                          : prec == 1 ? bf16x3_default_config(M, N, K)
                                      : f16s_default_config(M, N, K);
            std::printf("%d\n", c);
        } else if (op == 'E') {
            char ta, tb;
            long long M, N, K;
            in >> ta >> tb >> M >> N >> K;
            int64_t mm = -1, nn = -1;
            const bool split = f32_edge_plan(trans_code(ta) == 1, trans_code(tb) == 1, M, N, K,
                                             &mm, &nn);
            if (split) std::printf("1 %lld %lld\n", (long long)mm, (long long)nn);
            else std::printf("0 %lld %lld\n", (long long)mm, (long long)nn);
        } else if (op == 'T') {
            char ta, tb;
            long long M, N, K, lda, ldb, ldc;
            int cus;
            in >> ta >> tb >> M >> N >> K >> lda >> ldb >> ldc >> cus;
            const ThinPlan p = thin_plan(M, N, K, lda, ldb, ldc, trans_code(ta) == 1,
                                         trans_code(tb) == 1, cus);
            std::printf("%d %d %d %lld %lld %d\n", p.ok, p.rows, p.splits, (long long)p.kc,
                        (long long)thin_workspace_bytes(p, M, N, K), p.gather);
        } else if (op == 'S') {
            long long M, N, K;
            int cus;
            in >> M >> N >> K >> cus;
            const SplitKPlan p = f32_splitk_plan(M, N, K, cus);
            std::printf("%d %d %lld %lld\n", p.small_tile, p.splits, (long long)p.kc,
                        (long long)f32_splitk_workspace_bytes(p, M, N));
        } else if (op == 'L') {
            unsigned G;
            size_t n;
            in >> G >> n;
            std::vector<double> cost(n);
            for (double& c : cost) in >> c;
            const std::vector<uint32_t> owner = lpt_schedule(cost, G);
            for (size_t i = 0; i < owner.size(); ++i) std::printf(i ? " %u" : "%u", owner[i]);
            std::printf("\n");
        } else if (op == 'Q') {
            unsigned nq;
            size_t n;
            in >> nq >> n;
            std::vector<uint32_t> ntiles(n);
            std::vector<double> cost(n);
            for (uint32_t& t : ntiles) in >> t;
            for (double& c : cost) in >> c;
            const auto queues = queue_partition(ntiles, cost, nq);
            for (size_t q = 0; q < queues.size(); ++q) {
                std::printf(q ? " ; %zu" : "%zu", queues[q].size());
                for (const auto& pt : queues[q]) std::printf(" %u %u", pt.first, pt.second);
            }
            std::printf("\n");
        } else if (op == 'B') {
            size_t nc, na;
            in >> nc >> na;
            std::vector<Extent> cs(nc), ab(na);
            for (Extent& e : cs) in >> e.lo >> e.hi >> e.owner;
            for (Extent& e : ab) in >> e.lo >> e.hi >> e.owner;
            int kind = -1;
            const long long who = batch_alias(cs, ab, &kind);
            std::printf("%lld %d\n", who, kind);
        } else {
            std::printf("bad\n");
        }
    }
    return 0;
}
