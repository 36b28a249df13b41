// Host-side test of the table role lock (Sec. 3.5 compatibility table) with a recording event
// backend: threads issue calls of random roles on their own streams; afterwards the recorded
// stream orders and event edges must order every call after every call of the group before it,
// and must not order two calls of one group that ran on different streams.
//
//   roles_host_test <mode: 1 triple-group, 2 reader/writer> <threads> <calls per thread> <seed>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2603_17168_amd/csrc/cskv_roles.h"

struct Item {
    int kind;  // 0 call, 1 record, 2 wait
    int id;    // call index or event id
};

struct Log {
    std::mutex m;
    std::vector<std::vector<Item>> streams;
    int next_event = 0;
};

struct Recorder {
    using Event = int;
    using Stream = int;
    Log* L;
    Event make() {
        std::lock_guard<std::mutex> lk(L->m);
        return L->next_event++;
    }
    bool record(Event e, Stream s) {
        std::lock_guard<std::mutex> lk(L->m);
        L->streams[s].push_back({1, e});
        return true;
    }
    bool wait(Stream s, Event e) {
        std::lock_guard<std::mutex> lk(L->m);
        L->streams[s].push_back({2, e});
        return true;
    }
    bool done(Event) { return false; }  // never reused: every event id is unique
    void destroy(Event) {}
};

struct Call {
    int role;
    uint64_t group;
    int stream;
};

int main(int argc, char** argv) {
    if (argc != 5) return 2;
    const int mode = atoi(argv[1]), T = atoi(argv[2]), N = atoi(argv[3]);
    const unsigned seed = (unsigned)atoi(argv[4]);
    Log L;
    L.streams.resize(T);
    std::vector<Call> calls((size_t)T * N);
    {
        cskv::RoleLock<Recorder> lock(Recorder{&L});
        lock.set_mode(mode);
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t) {
            th.emplace_back([&, t] {
                std::mt19937 rng(seed * 7919u + (unsigned)t);
                for (int i = 0; i < N; ++i) {
                    const unsigned r = rng() % 10;
                    const int role = r < 5 ? cskv::kReader : (r < 8 ? cskv::kUpdater : cskv::kInserter);
                    const int id = t * N + i;
                    auto tk = lock.acquire(role, t);
                    {
                        std::lock_guard<std::mutex> lk(L.m);
                        L.streams[t].push_back({0, id});
                    }
                    calls[id] = Call{role, tk.seq, t};
                    if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
                    lock.release(tk, t);
                }
            });
        }
        for (auto& x : th) x.join();
    }
    // graph: nodes are the items of every stream; edges follow stream order and record -> wait
    std::vector<int> base(T + 1, 0);
    for (int t = 0; t < T; ++t) base[t + 1] = base[t] + (int)L.streams[t].size();
    const int nn = base[T];
    std::vector<std::vector<int>> out(nn);
    std::vector<int> rec_node(L.next_event, -1), call_node(calls.size(), -1);
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < (int)L.streams[t].size(); ++i) {
            const Item& it = L.streams[t][i];
            const int v = base[t] + i;
            if (i + 1 < (int)L.streams[t].size()) out[v].push_back(v + 1);
            if (it.kind == 1) rec_node[it.id] = v;
            if (it.kind == 0) call_node[it.id] = v;
        }
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < (int)L.streams[t].size(); ++i) {
            const Item& it = L.streams[t][i];
            if (it.kind == 2) {
                if (rec_node[it.id] < 0) {
                    printf("FAIL wait on an event never recorded\n");
                    return 1;
                }
                out[rec_node[it.id]].push_back(base[t] + i);
            }
        }
    // groups
    uint64_t ng = 0;
    for (const Call& c : calls) ng = std::max(ng, c.group);
    std::vector<std::vector<int>> members(ng + 1);
    for (int i = 0; i < (int)calls.size(); ++i) members[calls[i].group].push_back(i);
    long shared = 0;
    for (uint64_t g = 1; g <= ng; ++g) {
        const auto& m = members[g];
        if (m.empty()) {
            printf("FAIL empty group %llu\n", (unsigned long long)g);
            return 1;
        }
        for (int i : m)
            if (!cskv::roles_compatible(mode, calls[m[0]].role, calls[i].role) && m.size() > 1) {
                printf("FAIL incompatible calls share group %llu\n", (unsigned long long)g);
                return 1;
            }
        if (m.size() > 1) shared += (long)m.size();
    }
    std::vector<int> seen(nn, 0);
    int stamp = 0;
    auto reach = [&](int from) {
        ++stamp;
        std::vector<int> st{from};
        seen[from] = stamp;
        while (!st.empty()) {
            const int v = st.back();
            st.pop_back();
            for (int w : out[v])
                if (seen[w] != stamp) {
                    seen[w] = stamp;
                    st.push_back(w);
                }
        }
    };
    long ordered_pairs = 0, concurrent_pairs = 0;
    for (uint64_t g = 1; g <= ng; ++g)
        for (int a : members[g]) {
            reach(call_node[a]);
            if (g < ng)
                for (int b : members[g + 1]) {
                    if (seen[call_node[b]] != stamp) {
                        printf("FAIL call %d (group %llu) not ordered before call %d\n", a, (unsigned long long)g, b);
                        return 1;
                    }
                    ++ordered_pairs;
                }
            for (int b : members[g])
                if (b != a && calls[b].stream != calls[a].stream) {
                    if (seen[call_node[b]] == stamp) {
                        printf("FAIL calls %d and %d of group %llu are serialized\n", a, b, (unsigned long long)g);
                        return 1;
                    }
                    ++concurrent_pairs;
                }
        }
    printf("OK groups %llu calls %zu in shared groups %ld ordered pairs %ld concurrent pairs %ld events %d\n",
           (unsigned long long)ng, calls.size(), shared, ordered_pairs, concurrent_pairs, L.next_event);
    return 0;
}
