// Line-driven driver of the serving admission policy (serve_policy.h) for the
// CPU tests.  Commands on stdin, one per line:
//   reset SIZE                 empty arena of SIZE bytes, no pending requests
//   push TICKET GROUP BYTES    queue a request
//   form MAXB                  form one batch; prints
//                              "batch T:OFF ... blocked=T used=U ranges=R"
//   free TICKET                release a batched request's memory
//   bytes C H W                prints request_bytes(C, H, W)
//   state                      prints "used=U peak=P ranges=R pending=T,T,..."
#include <cstdio>
#include <iostream>
#include <map>
#include <sstream>
#include <string>

#include "serve_policy.h"

struct Req {
    uint64_t ticket = 0;
    int group = 0;
    size_t bytes = 0, off = 0;
};

int main() {
    qfca::serve::Arena arena;
    std::deque<Req> pending;
    std::map<uint64_t, Req> live;
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        std::string cmd;
        if (!(in >> cmd)) continue;
        if (cmd == "reset") {
            size_t n = 0;
            in >> n;
            arena.reset(n);
            pending.clear();
            live.clear();
        } else if (cmd == "push") {
            Req r;
            in >> r.ticket >> r.group >> r.bytes;
            pending.push_back(r);
        } else if (cmd == "form") {
            int maxb = 0;
            in >> maxb;
            std::vector<Req> out;
            uint64_t blocked = 0;
            qfca::serve::form_batch(pending, arena, maxb, out, &blocked);
            std::printf("batch");
            for (const Req& r : out) {
                std::printf(" %llu:%zu", (unsigned long long)r.ticket, r.off);
                live[r.ticket] = r;
            }
            std::printf(" blocked=%llu used=%zu ranges=%zu\n", (unsigned long long)blocked, arena.used(),
                        arena.free_ranges());
        } else if (cmd == "free") {
            uint64_t t = 0;
            in >> t;
            auto it = live.find(t);
            if (it == live.end()) {
                std::printf("error no such ticket\n");
                return 1;
            }
            arena.release(it->second.off, it->second.bytes);
            live.erase(it);
        } else if (cmd == "bytes") {
            int C = 0, H = 0, W = 0;
            in >> C >> H >> W;
            std::printf("%zu\n", qfca::serve::request_bytes(C, H, W));
        } else if (cmd == "state") {
            std::printf("used=%zu peak=%zu ranges=%zu pending=", arena.used(), arena.peak(), arena.free_ranges());
            for (size_t i = 0; i < pending.size(); ++i)
                std::printf(i ? ",%llu" : "%llu", (unsigned long long)pending[i].ticket);
            std::printf("\n");
        } else {
            std::printf("error unknown command\n");
            return 1;
        }
        std::fflush(stdout);
    }
    return 0;
}
